// Register-resident radix-16 Stockham FFT machinery shared by the time-axis
// transform kernels (single problem and batched).  A workgroup transforms W
// columns of length L; thread (t, c) holds P points of column c.  Between stages
// the points go through LDS one real plane at a time.
#pragma once
#include "aao_internal.h"

namespace aao {

// cos / sin of 2 pi k / 32 (double nearest)
constexpr double kC32[32] = {1, 0.980785280403230430579, 0.923879532511286738483, 0.831469612302545235671, 0.707106781186547572737, 0.555570233019602177649, 0.382683432365089781779, 0.195090322016128275839, 0.0, -0.195090322016128275839, -0.382683432365089781779, -0.555570233019602177649, -0.707106781186547572737, -0.831469612302545235671, -0.923879532511286738483, -0.980785280403230430579, -1, -0.980785280403230430579, -0.923879532511286738483, -0.831469612302545235671, -0.707106781186547572737, -0.555570233019602177649, -0.382683432365089781779, -0.195090322016128275839, 0.0, 0.195090322016128275839, 0.382683432365089781779, 0.555570233019602177649, 0.707106781186547572737, 0.831469612302545235671, 0.923879532511286738483, 0.980785280403230430579};
constexpr double kS32[32] = {0.0, 0.195090322016128275839, 0.382683432365089781779, 0.555570233019602177649, 0.707106781186547572737, 0.831469612302545235671, 0.923879532511286738483, 0.980785280403230430579, 1, 0.980785280403230430579, 0.923879532511286738483, 0.831469612302545235671, 0.707106781186547572737, 0.555570233019602177649, 0.382683432365089781779, 0.195090322016128275839, 0.0, -0.195090322016128275839, -0.382683432365089781779, -0.555570233019602177649, -0.707106781186547572737, -0.831469612302545235671, -0.923879532511286738483, -0.980785280403230430579, -1, -0.980785280403230430579, -0.923879532511286738483, -0.831469612302545235671, -0.707106781186547572737, -0.555570233019602177649, -0.382683432365089781779, -0.195090322016128275839};

// exp(-2 pi i k / 32) (conjugated when INV), k a compile-time constant after unrolling
template <bool INV, typename T>
__device__ __forceinline__ cx<T> root32(int k)
{
    k &= 31;
    return {T(kC32[k]), T(INV ? kS32[k] : -kS32[k])};
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
constexpr int bitrev(int v, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
    return r;
}

// In-register DFT of length R (1, 2, 4, 8 or 16):
//   v_s <- sum_r v_r exp(-+ 2 pi i r s / R)   (sign + when INV)
template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_reg(cx<T> *v)
{
    constexpr int LG = ilog2c(R);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int j = bitrev(i, LG);
        if (j > i) {
            cx<T> t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    }
#pragma unroll
    for (int m = 2; m <= R; m <<= 1) {
#pragma unroll
        for (int k = 0; k < R; k += m) {
#pragma unroll
            for (int jj = 0; jj < m / 2; ++jj) {
                const int ti = jj * (16 / m);      // index of exp(-2 pi i ti / 16)
                cx<T> b = v[k + jj + m / 2];
                cx<T> t;
                if (ti == 0) {
                    t = b;
                } else if (ti == 4) {               // multiply by -+ i
                    t = INV ? mul_i(b) : cx<T>{b.y, -b.x};
                } else {
                    t = root32<INV, T>(2 * ti) * b;
                }
                cx<T> a = v[k + jj];
                v[k + jj] = a + t;
                v[k + jj + m / 2] = a - t;
            }
        }
    }
}

// Stage plan of a length-L transform done with P points per thread: stages of
// radix RM = min(P, 16) and one smaller last stage if log2 L is not a multiple
// of log2 RM.
template <int L, int P> struct Plan {
    static constexpr int RM = P < 16 ? P : 16;
    static constexpr int LR = ilog2c(RM) > 0 ? ilog2c(RM) : 1;
    static constexpr int LG = ilog2c(L);
    static constexpr int NS = (LG + LR - 1) / LR;                 // number of stages
    static constexpr int radix(int s) {                           // RM,...,RM,rest
        return (s < NS - 1 || LG % LR == 0) ? RM : (1 << (LG % LR));
    }
    static constexpr int ns(int s) { return s == 0 ? 1 : ns(s - 1) * radix(s - 1); }
};

// Workgroups are dealt to the 8 XCDs round-robin (id mod 8).  Tiles that share
// 128-byte lines with their neighbours should meet in one XCD's L2, so the
// workgroup id is remapped to give each XCD a contiguous range of tiles.  The
// grid is padded to a multiple of 8; ids past the last tile map past n and idle.
__device__ __forceinline__ int xcd_tile(int g, int G)
{
    const int per = G / 8;
    return (g % 8) * per + g / 8;
}
__host__ __device__ constexpr int xcd_grid(int tiles) { return (tiles + 7) / 8 * 8; }

// LDS slot of (position, column): one padding row every 16 positions, so that
// the stride-16 position pattern of the first stage's outputs spreads the
// W-column groups of a wave over distinct banks.
__device__ __forceinline__ int lds_idx(int pos, int c, int W) { return (pos + (pos >> 4)) * W + c; }
__host__ __device__ constexpr int lds_rows(int L) { return L + L / 16 + 1; }

// Thread-held values: v[u*R + r] is input r of butterfly q = t + u*TN.
template <typename T, int L, int P, int S, bool INV>
__device__ __forceinline__ void stage_compute(cx<T> *v, int t, const cx<double> *tw, int twmul)
{
    constexpr int R = Plan<L, P>::radix(S);
    constexpr int NS_ = Plan<L, P>::ns(S);
    constexpr int TN = L / P;
#pragma unroll
    for (int u = 0; u < P / R; ++u) {
        if (NS_ > 1) {
            const int q = t + u * TN;
            const int k = q & (NS_ - 1);
            const int step = (L / (NS_ * R)) * twmul;   // twiddle w_{NS R}^{r k}
            // powers w^(2^b) from the table; w^r as the product over the set
            // bits of r (at most three roundings), so only log2(R) loads are live
            constexpr int LB = ilog2c(R);
            cx<T> wp[LB > 0 ? LB : 1];
#pragma unroll
            for (int b = 0; b < LB; ++b) {
                const cx<double> w = tw[(k << b) * step];
                wp[b] = {T(w.x), T(INV ? -w.y : w.y)};
            }
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<T> wt = {T(1), T(0)};
                bool first = true;
#pragma unroll
                for (int b = 0; b < LB; ++b)
                    if ((r >> b) & 1) {
                        wt = first ? wp[b] : wt * wp[b];
                        first = false;
                    }
                v[u * R + r] = wt * v[u * R + r];
            }
        }
        dft_reg<R, INV, T>(v + u * R);
    }
}

// Output position of value (u, r) after stage S.
template <int L, int P, int S>
__device__ __forceinline__ int out_pos(int t, int u, int r)
{
    constexpr int R = Plan<L, P>::radix(S);
    constexpr int NS_ = Plan<L, P>::ns(S);
    const int q = t + u * (L / P);
    return (q / NS_) * NS_ * R + (q & (NS_ - 1)) + r * NS_;
}

// Input position of value (u, r) before stage S.
template <int L, int P, int S>
__device__ __forceinline__ int in_pos(int t, int u, int r)
{
    constexpr int R = Plan<L, P>::radix(S);
    return t + u * (L / P) + r * (L / R);
}

// Exchange the outputs of stage S into the inputs of stage S+1 through LDS,
// one real plane at a time.
template <typename T, int L, int P, int S>
__device__ __forceinline__ void exchange(cx<T> *v, T *sm, int t, int c, int W)
{
    constexpr int R1 = Plan<L, P>::radix(S);
    constexpr int R2 = Plan<L, P>::radix(S + 1);
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
        for (int u = 0; u < P / R1; ++u)
#pragma unroll
            for (int r = 0; r < R1; ++r)
                sm[lds_idx(out_pos<L, P, S>(t, u, r), c, W)] = part ? v[u * R1 + r].y : v[u * R1 + r].x;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < P / R2; ++u)
#pragma unroll
            for (int r = 0; r < R2; ++r) {
                const T val = sm[lds_idx(in_pos<L, P, S + 1>(t, u, r), c, W)];
                if (part) v[u * R2 + r].y = val; else v[u * R2 + r].x = val;
            }
        __syncthreads();
    }
}

template <typename T, int L, int P, int S, bool INV>
__device__ __forceinline__ void run_stages(cx<T> *v, T *sm, int t, int c, int W,
                                           const cx<double> *tw, int twmul)
{
    if constexpr (S < Plan<L, P>::NS) {
        stage_compute<T, L, P, S, INV>(v, t, tw, twmul);
        if constexpr (S + 1 < Plan<L, P>::NS) {
            exchange<T, L, P, S>(v, sm, t, c, W);
            run_stages<T, L, P, S + 1, INV>(v, sm, t, c, W, tw, twmul);
        }
    }
}

// Position of held value idx after all stages (natural order).
template <int L, int P>
__device__ __forceinline__ int final_pos(int t, int idx)
{
    if constexpr (Plan<L, P>::NS == 0) {
        return 0;
    } else {
        constexpr int RL = Plan<L, P>::radix(Plan<L, P>::NS - 1);
        return out_pos<L, P, Plan<L, P>::NS - 1>(t, idx / RL, idx % RL);
    }
}
template <int L, int P>
__device__ __forceinline__ int first_pos(int t, int idx)
{
    if constexpr (Plan<L, P>::NS == 0) {
        return 0;
    } else {
        constexpr int R0 = Plan<L, P>::radix(0);
        return in_pos<L, P, 0>(t, idx / R0, idx % R0);
    }
}


}  // namespace aao
