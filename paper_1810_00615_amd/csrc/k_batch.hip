// Batched form: many independent all-at-once problems of uneven size (n_p, ell_p,
// kappa_p) advanced together, every phase of the preconditioned GMRES step as
// ONE launch over a table of work items that spans all problems (problem id and
// tile / row / slab).  Problems that have converged are masked out through a
// device flag, so the launch sequence of one Arnoldi step is fixed and can be
// captured in a hipGraph and replayed.
//
// The time-axis transform of a batch member uses Bluestein's chirp-z identity
// (jk = (j^2 + k^2 - (j-k)^2)/2), which turns a DFT of any length ell into a
// circular convolution of power-of-two length M >= 2 ell - 1, evaluated with
// the same register/LDS Stockham FFT as the single-problem path.  Two real
// columns travel as one complex sequence and are separated with the Hermitian
// symmetry of their spectra.
#include <algorithm>
#include <cstdlib>

#include <type_traits>

#include "batch.h"
#include "fft_core.h"
#include "lanes.h"
#include "solve_core.h"

namespace aao {

// Move values from the natural-order positions of a finished transform to the
// input positions of the first stage of the next one (both planes in turn).
template <typename T, int L, int P>
__device__ __forceinline__ void regroup(cx<T> *v, T *sm, int t, int c, int W)
{
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
        for (int idx = 0; idx < P; ++idx)
            sm[lds_idx(final_pos<L, P>(t, idx), c, W)] = part ? v[idx].y : v[idx].x;
        __syncthreads();
#pragma unroll
        for (int idx = 0; idx < P; ++idx) {
            const T val = sm[lds_idx(first_pos<L, P>(t, idx), c, W)];
            if (part) v[idx].y = val; else v[idx].x = val;
        }
        __syncthreads();
    }
}

template <typename T> __device__ __forceinline__ cx<T> cvt(cx<double> a) { return {T(a.x), T(a.y)}; }

// The second transform of a Bluestein tile reads the same twiddle and chirp
// entries as the first; left visible, the compiler keeps the first loads live
// across both transforms instead of loading again, and spills.  Offsetting the
// pointer by a zero the compiler cannot see through makes the loads repeat (an
// opaque offset rather than an opaque pointer, so that the global address space of
// the pointer is still known and the loads stay global loads, not flat ones).
template <typename P>
__device__ __forceinline__ P *fresh(P *p)
{
    int z = 0;
    asm volatile("" : "+s"(z));
    return p + z;
}

// ell <= M/2 always (M >= 2 ell - 1): the points of the first transform at positions
// >= M/2 are zero padding and the outputs of the second one there are never used.
// The position offset of a held value (its position at t = 0) is a compile-time
// constant after unrolling, so these tests let the compiler drop the zero inputs
// from the first stage and the unused outputs from the last one.
template <int M, int P>
__device__ __forceinline__ bool first_is_pad(int idx) { return first_pos<M, P>(0, idx) >= M / 2; }
template <int M, int P>
__device__ __forceinline__ bool final_is_unused(int idx) { return final_pos<M, P>(0, idx) >= M / 2; }

// Copy rows 0..ell-1, columns [cbase, cbase + C2) of a row-major ell x n array
// to LDS (row k at xs[k * C2], columns past n read as 0), and back.  ell <= M/2
// and C2 M = 2 NTB P, so both loops take exactly P passes of the NTB threads;
// the addresses are clamped so that every pass issues its load unconditionally.
template <int C2>
__device__ __forceinline__ void stage_rows(const double *__restrict__ rp, int n, int ell, int cbase,
                                           double *xs)
{
    constexpr int NQ = kBluesteinP, NTB = kBluesteinThreads;
    double val[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = threadIdx.x + u * NTB;
        const int k = min(q / C2, ell - 1), col = min(cbase + q % C2, n - 1);
        val[u] = rp[(size_t)k * n + col];
    }
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = threadIdx.x + u * NTB;
        const bool ok = q / C2 < ell && cbase + q % C2 < n;
        xs[q] = ok ? val[u] : 0.0;
    }
    __syncthreads();
}

template <int C2>
__device__ __forceinline__ void unstage_rows(const double *xs, int n, int ell, int cbase,
                                             double *__restrict__ zp)
{
    constexpr int NQ = kBluesteinP, NTB = kBluesteinThreads;
#pragma unroll 4   // (fully unrolled, the addresses of all eight stores spill)
    for (int u = 0; u < NQ; ++u) {
        const int q = threadIdx.x + u * NTB;
        const int k = q / C2, col = cbase + q % C2;
        if (k < ell && col < n) zp[(size_t)k * n + col] = xs[q];
    }
}

// Keep at most a few table loads in flight inside the fully unrolled per-point
// loops (the scheduler would otherwise hoist all of them and spill).
#define AAO_GROUP_FENCE(idx)                                     \
    do {                                                         \
        if (((idx) & 3) == 3) __builtin_amdgcn_sched_barrier(0); \
    } while (0)

// ---------------------------------------------------------- forward (Bluestein)
// X_j = c_j sum_k (x_k c_k) conj(c_{j-k}),  c_m = exp(-i pi m^2 / ell): the input
// a_k = x_k c_k is zero-padded to M, convolved with the filter through its
// precomputed spectrum, and the result multiplied by c_j.
template <typename T, int M>
__device__ void bl_fwd_tile(const BProb &pb, int tile, const double *__restrict__ r, double rs,
                            cx<T> *__restrict__ spec,
                            const cx<double> *__restrict__ chirp,
                            const cx<double> *__restrict__ bhat,
                            const cx<double> *__restrict__ twM, T *sm)
{
    constexpr int P = kBluesteinP;                    // points per thread
    constexpr int TN = M / P;
    constexpr int NTB = kBluesteinThreads;
    constexpr int W = NTB / TN;                       // column pairs per tile
    constexpr int C2 = 2 * W;                         // real columns per tile
    const int c = threadIdx.x % W;
    const int t = threadIdx.x / W;
    const int n = pb.n, ell = pb.ell;
    const int cbase = tile * C2;
    const double *rp = r + pb.off;
    const cx<double> *ch = chirp + pb.coff;
    // The tile's rows are staged in LDS first, C2 consecutive lanes reading one
    // row segment, so that every segment is one contiguous request (per-point
    // loads would touch each segment with several scattered requests).
    stage_rows<C2>(rp, n, ell, cbase, reinterpret_cast<double *>(sm));
    const double *xs = reinterpret_cast<const double *>(sm);
    cx<T> v[P];
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        const int k = first_pos<M, P>(t, idx);
        cx<T> a = {T(0), T(0)};
        if (!first_is_pad<M, P>(idx) && k < ell) {
            const double x0 = rs * xs[k * C2 + 2 * c], x1 = rs * xs[k * C2 + 2 * c + 1];
            const cx<double> ck = ch[k];
            a = cvt<T>(cx<double>{x0 * ck.x - x1 * ck.y, x0 * ck.y + x1 * ck.x});
        }
        v[idx] = a;
        AAO_GROUP_FENCE(idx);
    }
    __syncthreads();                                  // staging read before the first exchange
    run_stages<T, M, P, 0, false>(v, sm, t, c, W, twM, 4096 / M);
    const cx<double> *bh = bhat + pb.boff;           // spectrum of the forward filter
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        v[idx] = v[idx] * cvt<T>(bh[final_pos<M, P>(t, idx)]);
        AAO_GROUP_FENCE(idx);
    }
    regroup<T, M, P>(v, sm, t, c, W);
    run_stages<T, M, P, 0, true>(v, sm, t, c, W, fresh(twM), 4096 / M);
    // Z_j = c_j conv_j / M for j < ell; stage Z in LDS (complex) to pair j with ell-j
    const T invM = T(1.0 / M);
    const cx<double> *ch2 = fresh(ch);
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        const int j = final_pos<M, P>(t, idx);
        if (!final_is_unused<M, P>(idx) && j < ell) {
            const cx<T> z = cvt<T>(ch2[j]) * v[idx];
            sm[2 * (j * W + c)] = z.x * invM;
            sm[2 * (j * W + c) + 1] = z.y * invM;
        }
        AAO_GROUP_FENCE(idx);
    }
    __syncthreads();
    // X1_j = (Z_j + conj Z_{ell-j}) / 2,  X2_j = (Z_j - conj Z_{ell-j}) / 2i,  j <= ell/2;
    // consecutive lanes take consecutive columns of a spectrum row
    cx<T> *sp = spec + pb.soff;
    const int H = ell / 2;
    for (int q = threadIdx.x; q < (H + 1) * C2; q += NTB) {
        const int j = q / C2, cc = q % C2, pc = cc >> 1;
        const int jm = (ell - j) % ell;
        const cx<T> z = {sm[2 * (j * W + pc)], sm[2 * (j * W + pc) + 1]};
        const cx<T> zm = {sm[2 * (jm * W + pc)], sm[2 * (jm * W + pc) + 1]};
        // component-wise selects (a selected aggregate would be built in scratch)
        const bool second = cc & 1;
        const T ox = T(0.5) * (second ? z.y + zm.y : z.x + zm.x);
        const T oy = T(0.5) * (second ? zm.x - z.x : z.y - zm.y);
        if (cbase + cc < n) sp[(size_t)j * pb.lds + cbase + cc] = cx<T>{ox, oy};
    }
}

// ---------------------------------------------------------- inverse (Bluestein)
// x_k = (1/ell) conj(c_k) sum_j (Z_j conj(c_j)) c_{k-j}, Z = Y1 + i Y2 over the
// full spectrum (Y_{ell-j} = conj Y_j); Re x and Im x are the two real columns.
template <typename T, int M>
__device__ void bl_inv_tile(const BProb &pb, int tile, const cx<T> *__restrict__ spec,
                            double *__restrict__ z, const cx<double> *__restrict__ chirp,
                            const cx<double> *__restrict__ bhat,
                            const cx<double> *__restrict__ twM, T *sm)
{
    constexpr int P = kBluesteinP;
    constexpr int TN = M / P;
    constexpr int NTB = kBluesteinThreads;
    constexpr int W = NTB / TN;
    constexpr int C2 = 2 * W;                         // real columns per tile
    const int c = threadIdx.x % W;
    const int t = threadIdx.x / W;
    const int n = pb.n, ell = pb.ell;
    const int cbase = tile * C2;
    const cx<double> *ch = chirp + pb.coff;
    const cx<T> *sp = spec + pb.soff;
    const int H = ell / 2;
    // spectrum rows 0..H of the tile's columns staged in LDS, one contiguous
    // request per row segment
    // (H + 1) C2 <= (M/4 + 1) C2 = NTB P / 2 + C2 entries: P/2 + 1 passes, loads clamped
    cx<T> *ys = reinterpret_cast<cx<T> *>(sm);
    {
        constexpr int NQ = P / 2 + 1;
        T vx[NQ], vy[NQ];
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int q = threadIdx.x + u * NTB;
            const int j = min(q / C2, H), col = min(cbase + q % C2, n - 1);
            const cx<T> y = sp[(size_t)j * pb.lds + col];
            vx[u] = y.x;
            vy[u] = y.y;
        }
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int q = threadIdx.x + u * NTB;
            const bool in = cbase + q % C2 < n;
            if (q < (H + 1) * C2) ys[q] = cx<T>{in ? vx[u] : T(0), in ? vy[u] : T(0)};
        }
    }
    __syncthreads();
    cx<T> v[P];
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        const int j = first_pos<M, P>(t, idx);
        cx<T> a = {T(0), T(0)};
        if (!first_is_pad<M, P>(idx) && j < ell) {
            const bool up = j > H;
            const int jr = up ? ell - j : j;
            cx<T> y1 = ys[jr * C2 + 2 * c], y2 = ys[jr * C2 + 2 * c + 1];
            if (up) {
                y1 = conj(y1);
                y2 = conj(y2);
            }
            const cx<T> zz = y1 + mul_i(y2);
            a = zz * conj(cvt<T>(ch[j]));
        }
        v[idx] = a;
        AAO_GROUP_FENCE(idx);
    }
    __syncthreads();                                  // staging read before the first exchange
    run_stages<T, M, P, 0, false>(v, sm, t, c, W, twM, 4096 / M);
    const cx<double> *bh = bhat + pb.boff + M;       // spectrum of the inverse filter
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        v[idx] = v[idx] * cvt<T>(bh[final_pos<M, P>(t, idx)]);
        AAO_GROUP_FENCE(idx);
    }
    regroup<T, M, P>(v, sm, t, c, W);
    run_stages<T, M, P, 0, true>(v, sm, t, c, W, fresh(twM), 4096 / M);
    // rows of the result staged in LDS and written one contiguous segment per row
    const double scale = 1.0 / ((double)M * (double)ell);
    double *xs = reinterpret_cast<double *>(sm);
    const cx<double> *ch2 = fresh(ch);
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        const int k = final_pos<M, P>(t, idx);
        if (!final_is_unused<M, P>(idx) && k < ell) {
            const cx<T> x = conj(cvt<T>(ch2[k])) * v[idx];
            xs[k * C2 + 2 * c] = double(x.x) * scale;
            xs[k * C2 + 2 * c + 1] = double(x.y) * scale;
        }
        AAO_GROUP_FENCE(idx);
    }
    __syncthreads();
    unstage_rows<C2>(xs, n, ell, cbase, z + pb.off);
}

template <typename T>
// two workgroups per CU (at most 128 VGPRs), so that one can load or store
// while the other transforms
__global__ void __launch_bounds__(kBluesteinThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_batch_fft_fwd(const BProb *__restrict__ probs, const int2 *__restrict__ tiles, int ntiles,
                const unsigned char *__restrict__ active, const double *__restrict__ r,
                const double *__restrict__ scales, int sstride, cx<T> *__restrict__ spec, const cx<double> *__restrict__ chirp,
                const cx<double> *__restrict__ bhat, const cx<double> *__restrict__ twM)
{
    extern __shared__ unsigned char smraw[];
    T *sm = reinterpret_cast<T *>(smraw);
    const int g = xcd_tile(blockIdx.x, gridDim.x);
    if (g >= ntiles) return;
    const int2 e = tiles[g];
    if (active && !active[e.x]) return;
    const BProb pb = probs[e.x];
    const double rs = scales ? scales[(size_t)e.x * sstride] : 1.0;
    switch (pb.M) {
    case 512: bl_fwd_tile<T, 512>(pb, e.y, r, rs, spec, chirp, bhat, twM, sm); break;
    case 1024: bl_fwd_tile<T, 1024>(pb, e.y, r, rs, spec, chirp, bhat, twM, sm); break;
    case 2048: bl_fwd_tile<T, 2048>(pb, e.y, r, rs, spec, chirp, bhat, twM, sm); break;
    default: bl_fwd_tile<T, 4096>(pb, e.y, r, rs, spec, chirp, bhat, twM, sm); break;
    }
}

template <typename T>
// two workgroups per CU (at most 128 VGPRs), so that one can load or store
// while the other transforms
__global__ void __launch_bounds__(kBluesteinThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_batch_fft_inv(const BProb *__restrict__ probs, const int2 *__restrict__ tiles, int ntiles,
                const unsigned char *__restrict__ active, const cx<T> *__restrict__ spec,
                double *__restrict__ z, const cx<double> *__restrict__ chirp,
                const cx<double> *__restrict__ bhat, const cx<double> *__restrict__ twM)
{
    extern __shared__ unsigned char smraw[];
    T *sm = reinterpret_cast<T *>(smraw);
    const int g = xcd_tile(blockIdx.x, gridDim.x);
    if (g >= ntiles) return;
    const int2 e = tiles[g];
    if (active && !active[e.x]) return;
    const BProb pb = probs[e.x];
    switch (pb.M) {
    case 512: bl_inv_tile<T, 512>(pb, e.y, spec, z, chirp, bhat, twM, sm); break;
    case 1024: bl_inv_tile<T, 1024>(pb, e.y, spec, z, chirp, bhat, twM, sm); break;
    case 2048: bl_inv_tile<T, 2048>(pb, e.y, spec, z, chirp, bhat, twM, sm); break;
    default: bl_inv_tile<T, 4096>(pb, e.y, spec, z, chirp, bhat, twM, sm); break;
    }
}

// ------------------------------------------------------------ shifted solves
// Right-hand sides read from `in` (element type SI), solutions written to `out` (SO);
// in == out with SI == SO solves in place (a workgroup reads its row before writing).
template <typename A, typename SI, typename SO>
__global__ void __launch_bounds__(512)
k_batch_solve(const BProb *__restrict__ probs, const int2 *__restrict__ rows, int nrows,
              const unsigned char *__restrict__ active, const cx<SI> *in, cx<SO> *out,
              int scheme, int transpose, int *__restrict__ fail)
{
    constexpr int CW = 8;
    extern __shared__ unsigned char smraw[];
    const int NT = blockDim.x;
    cx<A> *tab = reinterpret_cast<cx<A> *>(smraw);
    cx<A> *red = tab + psolve_tab_entries(CW);
    cx<SI> *stage = reinterpret_cast<cx<SI> *>(red);
    cx<SO> *ostage = reinterpret_cast<cx<SO> *>(red);
    const int g = blockIdx.x;
    if (g >= nrows) return;
    const int2 e = rows[g];
    if (active && !active[e.x]) return;
    const BProb pb = probs[e.x];
    const int j = e.y, n = pb.n, ell = pb.ell, t = threadIdx.x;
    const cx<SI> *row = in + pb.soff + (size_t)j * pb.lds;
    cx<SO> *orow = out + pb.soff + (size_t)j * pb.lds;
    // heat: alpha = 1 - w^j, beta = tau;  BD2: alpha = (1 - w^j)^2, beta = tau^2
    double sn, cs;
    sincospi((transpose ? 2.0 : -2.0) * (double)j / (double)ell, &sn, &cs);
    double ar = 1.0 - cs, ai = -sn, br = pb.tau, bi = 0.0;
    if (scheme == 1) {
        const double r2 = ar * ar - ai * ai, i2 = 2.0 * ar * ai;
        ar = r2;
        ai = i2;
        br = pb.tau * pb.tau;
    }
    const double h = 1.0 / (n + 1.0), kap = pb.kappa;
    const cx<A> d = {A(ar * (4.0 * h / 6.0) + br * kap * (2.0 / h)), A(ai * (4.0 * h / 6.0) + bi * kap * (2.0 / h))};
    const cx<A> ee = {A(ar * (h / 6.0) - br * kap / h), A(ai * (h / 6.0) - bi * kap / h)};
    // odd row pitch: the chunk-wise and the coalesced accesses both spread over all banks
    const int NTP = NT + 1;
    const int ONTP = NT + 1;
    const int P = (n + CW - 1) / CW;
    const int len = (t < P) ? min(CW, n - t * CW) : 0;
    {
        // CW elements per thread (n <= CW NT), loaded together: unconditional at a
        // clamped index, parts kept apart (a whole-struct array would live in scratch)
        SI lx[CW], ly[CW];
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            const cx<SI> v = row[min(t + k * NT, n - 1)];
            lx[k] = v.x;
            ly[k] = v.y;
        }
#pragma unroll
        for (int k = 0; k < CW; ++k) {
            const int q = t + k * NT;
            if (q < n) stage[(q % CW) * NTP + q / CW] = {lx[k], ly[k]};
        }
    }
    __syncthreads();
    cx<A> y[CW];
#pragma unroll
    for (int i = 0; i < CW; ++i) {
        y[i] = {A(0), A(0)};
        if (i < len) {
            const cx<SI> v = stage[i * NTP + t];
            y[i] = {A(v.x), A(v.y)};
        }
    }
    const bool bad = partition_solve<A, CW>(y, n, d, ee, tab, red);
#pragma unroll
    for (int i = 0; i < CW; ++i)
        if (i < len) ostage[i * ONTP + t] = {SO(y[i].x), SO(y[i].y)};
    __syncthreads();
    for (int q = t; q < n; q += NT) orow[q] = ostage[(q % CW) * ONTP + q / CW];
    if (bad && fail) atomicOr(fail, 1);
}

// ------------------------------------------------------------------ matvec
// y = A x (or bsub - A x) per problem, tiles of 256 columns x RB time levels.  A
// thread loads its own column of each input row once; the i -+ 1 neighbours come
// from the adjacent lanes (DPP wave shift), and lanes 0 and 63 load the one
// neighbour outside their wave.  Threads past n stay for the lane moves (with 0).
//
// DOTS > 0: the tile also leaves the partials of V_q . y, q < DOTS (the first
// Gram-Schmidt pass of an early Arnoldi step), at part[tile * ldp + q]; DOTS = -1:
// the partial of y . y (the norm of a residual), from registers.
template <int DOTS, int RB>
__global__ void __launch_bounds__(256)
k_batch_matvec(const BProb *__restrict__ probs, const int4 *__restrict__ tiles, int ntiles,
               const unsigned char *__restrict__ active, const double *__restrict__ x,
               double *__restrict__ y, const double *__restrict__ bsub, int scheme, int transpose,
               const double *const *__restrict__ Vd, double *__restrict__ part, int ldp)
{
    constexpr int ND = DOTS < 0 ? 1 : DOTS;        // partials per tile
    __shared__ double red[(ND > 0 ? ND : 1) * 4];
    const int g = blockIdx.x;
    if (g >= ntiles) return;
    const int4 e = tiles[g];
    if (active && !active[e.x]) return;
    const BProb pb = probs[e.x];
    const int n = pb.n, ell = pb.ell;
    const int lane = threadIdx.x & 63;
    const int i = e.y * 256 + threadIdx.x;
    const bool col = i < n;
    const int je = lane == 0 ? i - 1 : i + 1;        // outside neighbour of lanes 0 / 63
    const bool edge = (lane == 0 || lane == 63) && je >= 0 && je < n;
    const int s = scheme == 1 ? 2 : 1;
    double am[3], bm[3];
    if (scheme == 1) {
        am[0] = 1.0; am[1] = -2.0; am[2] = 1.0;
        bm[0] = pb.tau * pb.tau * pb.kappa; bm[1] = 0.0; bm[2] = 0.0;
    } else {
        am[0] = 1.0; am[1] = -1.0; am[2] = 0.0;
        bm[0] = pb.tau * pb.kappa; bm[1] = 0.0; bm[2] = 0.0;
    }
    const double h = 1.0 / (n + 1.0);
    const int k0 = e.z * RB, k1 = min(k0 + RB, ell);
    const int nin = (k1 - k0) + s;
    const double *xp = x + pb.off;
    constexpr int NR = RB + 2;
    double rl[NR], rc[NR], rr[NR];
#pragma unroll
    for (int it = 0; it < NR; ++it) {
        const int kk = transpose ? (k1 - 1 + s - it) : (k0 - s + it);
        const bool in = it < nin && kk >= 0 && kk < ell;
        const double *row = xp + (size_t)(in ? kk : 0) * n;
        rc[it] = (in && col) ? row[i] : 0.0;
        rr[it] = (in && edge) ? row[je] : 0.0;      // edge value, replaced below
    }
#pragma unroll
    for (int it = 0; it < NR; ++it) {
        const double l = lane_from_left<true>(rc[it]);
        const double r = lane_from_right<true>(rc[it]);
        const double ev = rr[it];
        rl[it] = lane == 0 ? ev : l;
        rr[it] = lane == 63 ? ev : r;
    }
    if (DOTS == 0 && !col) return;
    double acc[ND > 0 ? ND : 1] = {};
    if (col) {
#pragma unroll
        for (int it = 0; it < NR; ++it) {
            if (it < s || it >= nin) continue;
            const int k = transpose ? (k1 - 1 + s - it) : (k0 - s + it);
            double al = 0, ac = 0, ar = 0, bl = 0, bc = 0, br = 0;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                if (m > s || it - m < 0) break;
                al += am[m] * rl[it - m];
                ac += am[m] * rc[it - m];
                ar += am[m] * rr[it - m];
                bl += bm[m] * rl[it - m];
                bc += bm[m] * rc[it - m];
                br += bm[m] * rr[it - m];
            }
            const double v = (h / 6.0) * (al + 4.0 * ac + ar) + (1.0 / h) * (2.0 * bc - bl - br);
            const size_t o = pb.off + (size_t)k * n + i;
            const double out = bsub ? bsub[o] - v : v;
            y[o] = out;
            if constexpr (DOTS < 0) {
                acc[0] += out * out;
            } else {
#pragma unroll
                for (int q = 0; q < DOTS; ++q) acc[q] += Vd[q][o] * out;
            }
        }
    }
    if constexpr (ND > 0) {
#pragma unroll
        for (int q = 0; q < ND; ++q) {
            double v = acc[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) red[q * 4 + (threadIdx.x >> 6)] = v;
        }
        __syncthreads();
        if (threadIdx.x < ND)
            part[(size_t)g * ldp + threadIdx.x] = red[threadIdx.x * 4] + red[threadIdx.x * 4 + 1] +
                                                  red[threadIdx.x * 4 + 2] + red[threadIdx.x * 4 + 3];
    }
}

// ------------------------------------------------- Gram-Schmidt (per problem)
// Each block owns one slab of one problem.  MODE 0: dots of the nv basis
// vectors with w; MODE 1: w' = w - sum V_i c_i, dots with w'; MODE 2:
// w'' = w - sum V_i c_i written to out, and ||w''||^2.  Coefficients c are per
// problem (c[p * cst + i]).  Partials: part[slab * ldp + slot].
//
// MODE 3 (CGS2 with the re-orthogonalisation deferred by one step): V_0..V_{j-1}
// hold the final basis (V_0 with its scale folded into the coefficients), V_j the
// pending vector p_j (j = nv - 1).  Per element, v_j = s p_j - sum_{i<j} a_i V_i
// (s = coef[kBC - 2], a_i = coef2[i]) is written over p_j when j > 0, and
// w1 = w - sum_{i<j} c_i V_i - h_j v_j (c_i = coef[i], h_j = coef[kBC - 1]) to out;
// the partials are V_i . w1 (slots i < j), v_j . w1 (slot j) and w1 . w1 (slot nv).
constexpr int kBC = kBSmall;   // coefficients per problem (the small arrays' stride)

template <int MODE, int NV>
__global__ void __launch_bounds__(256)
k_batch_cgs(const BProb *__restrict__ probs, const int4 *__restrict__ slabs, int nslabs,
            const unsigned char *__restrict__ active, const double *const *__restrict__ V, int nv,
            const double *__restrict__ w, const double *__restrict__ coef, int cst,
            double *__restrict__ out, double *__restrict__ part, int ldp,
            const double *__restrict__ coef2 = nullptr)
{
    __shared__ double red[(NV + 1) * 4];
    const int g = blockIdx.x;
    if (g >= nslabs) return;
    const int4 e = slabs[g];                      // (problem, first, count, -)
    const bool act = !active || active[e.x];
    double acc[NV + 1];
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
    if (act) {
        const size_t base = probs[e.x].off + (size_t)e.y;
        const int j = nv - 1;
        double cf[NV], ca[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const bool use = MODE == 3 ? i < j : (MODE > 0 && i < nv);
            cf[i] = use ? coef[(size_t)e.x * cst + i] : 0.0;
            ca[i] = (MODE == 3 && i < j) ? coef2[(size_t)e.x * cst + i] : 0.0;
        }
        const double sp = MODE == 3 ? coef[(size_t)e.x * cst + kBC - 2] : 0.0;
        const double hj = MODE == 3 ? coef[(size_t)e.x * cst + kBC - 1] : 0.0;
        // the pending vector is workspace storage when j > 0 (V_0 may be the caller's b)
        double *pj = (MODE == 3 && j > 0) ? const_cast<double *>(V[j]) : nullptr;
        // a norm (the only vector is w itself) reads w once
        const bool self = MODE == 0 && nv == 1 && V[0] == w;
        for (int q = threadIdx.x; q < e.z; q += blockDim.x) {
            const size_t o = base + q;
            double s = w[o];
            double vv[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) vv[i] = (i < nv && !(i == 0 && self)) ? V[i][o] : 0.0;
            if (self) vv[0] = s;
            if (MODE == 3) {
                double vj = 0.0;
#pragma unroll
                for (int i = 0; i < NV; ++i)
                    if (i == j) vj = sp * vv[i];
#pragma unroll
                for (int i = 0; i < NV; ++i) vj -= ca[i] * vv[i];
#pragma unroll
                for (int i = 0; i < NV; ++i) s -= cf[i] * vv[i];
                s -= hj * vj;
                if (pj) pj[o] = vj;
                out[o] = s;
#pragma unroll
                for (int i = 0; i < NV; ++i) acc[i] += (i < j ? vv[i] : (i == j ? vj : 0.0)) * s;
                acc[NV] += s * s;
            } else if (MODE == 0) {
#pragma unroll
                for (int i = 0; i < NV; ++i) acc[i] += vv[i] * s;
            } else {
#pragma unroll
                for (int i = 0; i < NV; ++i) s -= vv[i] * cf[i];
                if (MODE == 1) {
#pragma unroll
                    for (int i = 0; i < NV; ++i) acc[i] += vv[i] * s;
                } else {
                    out[o] = s;
                    acc[NV] += s * s;
                }
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i <= NV; ++i) {
        const bool used = (i < NV) ? (MODE != 2 && i < nv) : (MODE >= 2);
        if (used) {
            double v = acc[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) red[i * 4 + wv] = v;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= NV; i += blockDim.x) {
        const bool used = (i < NV) ? (MODE != 2 && i < nv) : (MODE >= 2);
        if (!used) continue;
        const double sum = red[i * 4] + red[i * 4 + 1] + red[i * 4 + 2] + red[i * 4 + 3];
        part[(size_t)g * ldp + (i < NV ? i : (MODE == 3 ? nv : 0))] = sum;
    }
}

// sums[p * sst + i] = sum over the slabs of problem p of part[slab * ldp + i]
__global__ void k_batch_reduce(const int2 *__restrict__ pslabs, int count,
                               const unsigned char *__restrict__ active,
                               const double *__restrict__ part, int ldp, int cnt,
                               double *__restrict__ sums, int sst)
{
    // one wave per (problem, value): lane l sums blocks l, l + 64, ... in order (eight
    // loads in flight), then a fixed shuffle tree (the order is the same on every run)
    const int p = blockIdx.x, i = blockIdx.y;
    if (p >= count || i >= cnt || (active && !active[p])) return;
    const int2 rg = pslabs[p];                     // block range [x, y)
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int b0 = rg.x; b0 < rg.y; b0 += 8 * 64) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int b = b0 + k * 64 + lane;
            v[k] = b < rg.y ? part[(size_t)b * ldp + i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) sums[(size_t)p * sst + i] = s;
}

// Per-problem Arnoldi bookkeeping and Givens update, one thread per problem.
//   mode 0: h1 = vs.d, c = vs.h1
//   mode 1: h2 = vs.d, c += vs.h2
//   mode 2: nrm = sqrt(d0); vs[j+1] = 1/nrm; H column = [h1 + h2, nrm]; apply the
//           previous rotations, form rotation j, update g, test convergence
//   mode 3: restart vector: nrm = sqrt(d0) = beta; vs[0] = 1/beta; g = [beta, 0..];
//           active = (beta / bnorm > tol) && !done
//   mode 4: (deferred CGS2, after the dots of w with V_0..V_j) the column's h_i and
//           the coefficients of the update pass
//   mode 5: (after the update pass) the re-orthogonalisation coefficients of the new
//           pending vector, the completed column, scales, Givens and convergence
template <int dummy>
__global__ void k_batch_small(int mode, int count, int j, int m, double tol, BState st)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    if (mode != 3 && !st.active[p]) return;
    const int nv = j + 1;
    double *d = st.dsum + (size_t)p * st.sst;
    double *h1 = st.h1 + (size_t)p * st.sst;
    double *h2 = st.h2 + (size_t)p * st.sst;
    double *c = st.coef + (size_t)p * st.sst;
    double *vs = st.vs + (size_t)p * st.sst;
    if (mode == 0) {
        for (int i = 0; i < nv; ++i) {
            h1[i] = vs[i] * d[i];
            c[i] = vs[i] * h1[i];
        }
    } else if (mode == 1) {
        for (int i = 0; i < nv; ++i) {
            h2[i] = vs[i] * d[i];
            c[i] += vs[i] * h2[i];
        }
    } else if (mode == 2) {
        const double nrm = sqrt(fmax(d[0], 0.0));
        vs[nv] = nrm > 0.0 ? 1.0 / nrm : 0.0;
        double *H = st.H + (size_t)p * st.hst;          // column-major (m+1) x m
        double *hc = H + (size_t)j * (m + 1);
        for (int i = 0; i < nv; ++i) hc[i] = h1[i] + h2[i];
        hc[nv] = nrm;
        double *cs = st.cs + (size_t)p * st.sst, *sn = st.sn + (size_t)p * st.sst;
        double *gg = st.g + (size_t)p * st.sst;
        for (int i = 0; i < j; ++i) {
            const double a = cs[i] * hc[i] + sn[i] * hc[i + 1];
            hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
            hc[i] = a;
        }
        const double den = hypot(hc[j], hc[j + 1]);
        const bool ok = den > 0.0 && isfinite(den);
        cs[j] = ok ? hc[j] / den : 1.0;
        sn[j] = ok ? hc[j + 1] / den : 0.0;
        hc[j] = ok ? den : hc[j];
        hc[j + 1] = 0.0;
        gg[j + 1] = -sn[j] * gg[j];
        gg[j] = cs[j] * gg[j];
        st.iters[p] += 1;
        st.ksteps[p] = nv;
        const double est = fabs(gg[j + 1]) / st.bnorm[p];
        st.est[p] = est;
        if (!ok || !(est > tol) || st.iters[p] >= st.maxit) st.active[p] = 0;
        if (!ok || !isfinite(est)) st.bad[p] = 1;
    } else if (mode == 4 || mode == 5) {
        // CGS2 with the re-orthogonalisation deferred by one step.  h2[0..j-1] and
        // h2[kBC-1] hold the coefficients a_i and alpha of the pending p_j (unit after
        // the scale vs[j]): p_j vs_j = sum_{i<j} a_i v_i + alpha v_j.
        double *H = st.H + (size_t)p * st.hst;          // column-major (m+1) x m
        double *hc = H + (size_t)j * (m + 1);
        double *a = h2;
        if (mode == 4) {
            // d_i = V_i . w (i < j: final basis, v_i = vs_i V_i), d_j = p_j . w
            const double alpha = j > 0 ? a[kBC - 1] : 1.0;
            double hj = vs[j] * d[j];
            for (int i = 0; i < j; ++i) {
                hc[i] = vs[i] * d[i];
                hj -= a[i] * hc[i];
                c[i] = hc[i] * vs[i];                    // w1 coefficients on V_i
                h1[i] = a[i] * vs[i] / alpha;            // v_j = (vs_j p_j - sum a_i v_i) / alpha
            }
            hj /= alpha;
            hc[j] = hj;
            c[kBC - 2] = vs[j] / alpha;
            c[kBC - 1] = hj;
        } else {
            // d_i = V_i . w1 (i < j), d_j = v_j . w1, d_nv = w1 . w1
            const double nrm = sqrt(fmax(d[nv], 0.0));
            const double sn1 = nrm > 0.0 ? 1.0 / nrm : 0.0;
            double aa = 0.0;
            for (int i = 0; i <= j; ++i) {
                const double ai = (i < j ? vs[i] : 1.0) * d[i] * sn1;
                a[i] = ai;
                aa += ai * ai;
                hc[i] += nrm * ai;
            }
            const double alpha = sqrt(fmax(1.0 - aa, 0.0));
            a[kBC - 1] = alpha;
            hc[nv] = nrm * alpha;
            if (j > 0) vs[j] = 1.0;                      // v_j now stored normalised
            vs[nv] = sn1;                                // scale of the pending p_{j+1}
            double *cs = st.cs + (size_t)p * st.sst, *sn = st.sn + (size_t)p * st.sst;
            double *gg = st.g + (size_t)p * st.sst;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
                hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
                hc[i] = t;
            }
            const double den = hypot(hc[j], hc[j + 1]);
            const bool ok = den > 0.0 && isfinite(den);
            cs[j] = ok ? hc[j] / den : 1.0;
            sn[j] = ok ? hc[j + 1] / den : 0.0;
            hc[j] = ok ? den : hc[j];
            hc[j + 1] = 0.0;
            gg[j + 1] = -sn[j] * gg[j];
            gg[j] = cs[j] * gg[j];
            st.iters[p] += 1;
            st.ksteps[p] = nv;
            const double est = fabs(gg[j + 1]) / st.bnorm[p];
            st.est[p] = est;
            if (!ok || !(est > tol) || st.iters[p] >= st.maxit) st.active[p] = 0;
            if (!ok || !isfinite(est)) st.bad[p] = 1;
        }
    } else {
        const double beta = sqrt(fmax(d[0], 0.0));
        vs[0] = beta > 0.0 ? 1.0 / beta : 0.0;
        double *gg = st.g + (size_t)p * st.sst;
        gg[0] = beta;
        st.ksteps[p] = 0;
        const double rel = beta / st.bnorm[p];
        st.truer[p] = rel;
        if (!isfinite(rel)) st.bad[p] = 1;
        const bool conv = !(rel > tol);
        st.done[p] = conv ? 1 : st.done[p];
        st.active[p] = (!conv && st.iters[p] < st.maxit && !st.bad[p]) ? 1 : 0;
    }
}

// y = R^{-1} g per problem (k steps), one thread per problem
__global__ void k_batch_backsolve(int count, int m, BState st)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    const int k = st.ksteps[p];
    const double *H = st.H + (size_t)p * st.hst;
    const double *gg = st.g + (size_t)p * st.sst;
    double *y = st.y + (size_t)p * st.sst;
    for (int i = k - 1; i >= 0; --i) {
        double s = gg[i];
        for (int l = i + 1; l < k; ++l) s -= H[(size_t)l * (m + 1) + i] * y[l];
        y[i] = s / H[(size_t)i * (m + 1) + i];
    }
}

// x += sum_{i < k_p} Z_i y_i per problem, over slabs (x = sum ... when overwrite).
// KM >= every k_p: the direction loop is unrolled, so the loads of one element are
// all in flight together.
template <int KM>
__global__ void __launch_bounds__(256)
k_batch_axpy(const BProb *__restrict__ probs, const int4 *__restrict__ slabs, int nslabs,
             const double *const *__restrict__ Z, BState st, double *__restrict__ x, int overwrite)
{
    const int g = blockIdx.x;
    if (g >= nslabs) return;
    const int4 e = slabs[g];
    const int k = st.ksteps[e.x];
    if (k == 0 && !overwrite) return;
    const double *y = st.y + (size_t)e.x * st.sst;
    double yc[KM];
    const double *zp[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) {
        yc[i] = i < k ? y[i] : 0.0;
        zp[i] = Z[i < k ? i : 0];
    }
    const size_t base = probs[e.x].off + (size_t)e.y;
    for (int q = threadIdx.x; q < e.z; q += blockDim.x) {
        const size_t o = base + q;
        double s = overwrite ? 0.0 : x[o];
        // unconditional loads (directions past k_p read Z_0, valid workspace) and
        // a select, so that no branch separates the loads
        double zv[KM];
#pragma unroll
        for (int i = 0; i < KM; ++i) zv[i] = zp[i][o];
#pragma unroll
        for (int i = 0; i < KM; ++i) s += i < k ? zv[i] * yc[i] : 0.0;
        x[o] = s;
    }
}

__global__ void k_batch_copy_active(const unsigned char *__restrict__ a, int count,
                                    int *__restrict__ nact)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int s = 0;
    for (int p = 0; p < count; ++p) s += a[p] ? 1 : 0;
    *nact = s;
}

// ----------------------------------------------------------------- setup
// chirp c_m = exp(-i pi m^2 / ell) with m^2 reduced mod 2 ell in integers
__global__ void k_batch_chirp(const BProb *__restrict__ probs, int count,
                              cx<double> *__restrict__ chirp)
{
    const int p = blockIdx.y;
    if (p >= count) return;
    const BProb pb = probs[p];
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < pb.ell; m += gridDim.x * blockDim.x) {
        const long long q = ((long long)m * m) % (2LL * pb.ell);
        double s, c;
        sincospi(-(double)q / (double)pb.ell, &s, &c);
        chirp[pb.coff + m] = {c, s};
    }
}

// Filter spectra by a direct DFT of length M (setup only):
//   forward filter  b_m = conj(c_m), |m| < ell (wrapped), inverse filter c_m.
// Filter spectra of a problem: the forward filter b_m = conj(c_m) (m < ell) and
// conj(c_{M-m}) (m > M - ell), zero between (M >= 2 ell - 1), is even in m, so its
// length-M DFT is B_q = conj(c_0) + 2 sum_{m=1}^{ell-1} conj(c_m) cos(2 pi q m / M); the
// inverse filter's (c in place of conj c) is conj(B_q).  The cosines come from a
// table of the M-th roots in LDS (exact index q m mod M), one workgroup row of q.
__global__ void __launch_bounds__(256)
k_batch_bhat(const BProb *__restrict__ probs, int count, const cx<double> *__restrict__ chirp,
             cx<double> *__restrict__ bhat)
{
    __shared__ double cosq[4096];
    const int p = blockIdx.y;
    if (p >= count) return;
    const BProb pb = probs[p];
    const int M = pb.M, ell = pb.ell;
    if ((int)blockIdx.x * (int)blockDim.x >= M) return;   // (uniform over the workgroup)
    for (int k = threadIdx.x; k < M; k += blockDim.x) cosq[k] = cospi(2.0 * k / (double)M);
    __syncthreads();
    const cx<double> *ch = chirp + pb.coff;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    double fr = 0.0, fi = 0.0;
    for (int m = 1; m < ell; ++m) {
        const double cs = cosq[(int)(((long long)q * m) & (M - 1))];
        const cx<double> cm = ch[m];
        fr += cm.x * cs;
        fi -= cm.y * cs;
    }
    const cx<double> c0 = ch[0];
    fr = c0.x + 2.0 * fr;
    fi = -c0.y + 2.0 * fi;
    bhat[pb.boff + q] = {fr, fi};
    bhat[pb.boff + M + q] = {fr, -fi};
}

// ------------------------------------------------------------- launchers
hipError_t bl_twiddles(double *tw, hipStream_t st) { return launch_twiddles(tw, 4096, 4096, st); }

hipError_t batch_setup_tables(const BProb *probs, int count, int max_ell, int max_M,
                              double *chirp, double *bhat, hipStream_t st)
{
    dim3 g1((max_ell + 255) / 256, count);
    k_batch_chirp<<<g1, 256, 0, st>>>(probs, count, reinterpret_cast<cx<double> *>(chirp));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2((max_M + 255) / 256, count);
    k_batch_bhat<<<g2, 256, 0, st>>>(probs, count, reinterpret_cast<const cx<double> *>(chirp),
                                     reinterpret_cast<cx<double> *>(bhat));
    return hipGetLastError();
}

static size_t bl_smem(size_t realsz)
{
    // largest of, over M in {512..4096} (W = NTB P / M pairs, C2 = 2 W columns,
    // ell <= M/2): the tile plane lds_rows(M) W reals; the staged real rows
    // ell C2 doubles; the staged spectrum rows (M/4 + 1) C2 complex values
    size_t best = 0;
    for (int M = 512; M <= 4096; M *= 2) {
        const size_t W = bluestein_pairs(M), C2 = 2 * W;
        const size_t plane = (size_t)lds_rows(M) * W * realsz;
        const size_t rows = (size_t)(M / 2) * C2 * sizeof(double);
        const size_t spec = (size_t)(M / 4 + 1) * C2 * 2 * realsz;
        best = std::max(best, std::max(plane, std::max(rows, spec)));
    }
    return best;
}

static size_t solve_smem(size_t es, size_t as, int NT = 512)
{
    const int CW = 8;
    const size_t stage = es * CW * (NT + 4), redb = as * 6 * NT;
    return as * psolve_tab_entries(CW) + (stage > redb ? stage : redb);
}

// Dynamic-LDS limits of the batched kernels, set once before any graph capture.
hipError_t batch_prepare()
{
    hipError_t e;
#define AAO_ATTR(k, bytes)                                                                     \
    e = hipFuncSetAttribute((const void *)(k), hipFuncAttributeMaxDynamicSharedMemorySize,      \
                            (int)(bytes));                                                    \
    if (e != hipSuccess) return e;
    AAO_ATTR(k_batch_fft_fwd<float>, bl_smem(sizeof(float)))
    AAO_ATTR(k_batch_fft_fwd<double>, bl_smem(sizeof(double)))
    AAO_ATTR(k_batch_fft_inv<float>, bl_smem(sizeof(float)))
    AAO_ATTR(k_batch_fft_inv<double>, bl_smem(sizeof(double)))
    AAO_ATTR((k_batch_solve<double, double, double>), solve_smem(16, 16))
    AAO_ATTR((k_batch_solve<double, float, float>), solve_smem(8, 16))
    AAO_ATTR((k_batch_solve<float, float, float>), solve_smem(8, 8))
    AAO_ATTR((k_batch_solve<double, float, double>), solve_smem(16, 16))
#undef AAO_ATTR
    return hipSuccess;
}

hipError_t batch_fft_fwd(const BatchLaunch &L, const double *r, const double *scales, int sstride,
                         void *spec, bool single, hipStream_t st)
{
    const int G = xcd_grid(L.nftiles);
    if (single) {
        const size_t smem = bl_smem(sizeof(float));
        auto k = k_batch_fft_fwd<float>;
        k<<<G, kBluesteinThreads, smem, st>>>(L.probs, L.ftiles, L.nftiles, L.active, r, scales, sstride,
                                 reinterpret_cast<cx<float> *>(spec),
                                 reinterpret_cast<const cx<double> *>(L.chirp),
                                 reinterpret_cast<const cx<double> *>(L.bhat),
                                 reinterpret_cast<const cx<double> *>(L.tw));
    } else {
        const size_t smem = bl_smem(sizeof(double));
        auto k = k_batch_fft_fwd<double>;
        k<<<G, kBluesteinThreads, smem, st>>>(L.probs, L.ftiles, L.nftiles, L.active, r, scales, sstride,
                                 reinterpret_cast<cx<double> *>(spec),
                                 reinterpret_cast<const cx<double> *>(L.chirp),
                                 reinterpret_cast<const cx<double> *>(L.bhat),
                                 reinterpret_cast<const cx<double> *>(L.tw));
    }
    return hipGetLastError();
}

hipError_t batch_fft_inv(const BatchLaunch &L, const void *spec, double *z, bool single,
                         hipStream_t st)
{
    const int G = xcd_grid(L.nftiles);
    if (single) {
        const size_t smem = bl_smem(sizeof(float));
        auto k = k_batch_fft_inv<float>;
        k<<<G, kBluesteinThreads, smem, st>>>(L.probs, L.ftiles, L.nftiles, L.active,
                                 reinterpret_cast<const cx<float> *>(spec), z,
                                 reinterpret_cast<const cx<double> *>(L.chirp),
                                 reinterpret_cast<const cx<double> *>(L.bhat),
                                 reinterpret_cast<const cx<double> *>(L.tw));
    } else {
        const size_t smem = bl_smem(sizeof(double));
        auto k = k_batch_fft_inv<double>;
        k<<<G, kBluesteinThreads, smem, st>>>(L.probs, L.ftiles, L.nftiles, L.active,
                                 reinterpret_cast<const cx<double> *>(spec), z,
                                 reinterpret_cast<const cx<double> *>(L.chirp),
                                 reinterpret_cast<const cx<double> *>(L.bhat),
                                 reinterpret_cast<const cx<double> *>(L.tw));
    }
    return hipGetLastError();
}

hipError_t batch_solve(const BatchLaunch &L, const void *in, void *out, bool single_in,
                       bool single_out, bool single_arith, int scheme, int transpose, int *fail,
                       hipStream_t st)
{
    if ((in == out && single_in != single_out) || (single_arith && !(single_in && single_out)) ||
        (!single_in && single_out))
        return hipErrorInvalidValue;
    // one launch per class of n: NT = 64 << c threads cover n <= 8 NT unknowns
    for (int c = 0; c < kSolveClasses; ++c) {
        const int first = L.row_start[c], count = L.row_start[c + 1] - first;
        if (count <= 0) continue;
        const int NT = 64 << c;
        const int2 *rows = L.rows + first;
        if (!single_in) {
            k_batch_solve<double, double, double><<<count, NT, solve_smem(16, 16, NT), st>>>(
                L.probs, rows, count, L.active, reinterpret_cast<const cx<double> *>(in),
                reinterpret_cast<cx<double> *>(out), scheme, transpose, fail);
        } else if (!single_out) {
            k_batch_solve<double, float, double><<<count, NT, solve_smem(16, 16, NT), st>>>(
                L.probs, rows, count, L.active, reinterpret_cast<const cx<float> *>(in),
                reinterpret_cast<cx<double> *>(out), scheme, transpose, fail);
        } else if (!single_arith) {
            k_batch_solve<double, float, float><<<count, NT, solve_smem(8, 16, NT), st>>>(
                L.probs, rows, count, L.active, reinterpret_cast<const cx<float> *>(in),
                reinterpret_cast<cx<float> *>(out), scheme, transpose, fail);
        } else {
            k_batch_solve<float, float, float><<<count, NT, solve_smem(8, 8, NT), st>>>(
                L.probs, rows, count, L.active, reinterpret_cast<const cx<float> *>(in),
                reinterpret_cast<cx<float> *>(out), scheme, transpose, fail);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t batch_matvec(const BatchLaunch &L, const double *x, double *y, const double *bsub,
                        int scheme, int transpose, bool masked, hipStream_t st,
                        const double *const *Vd, int nd, double *part, int ldp)
{
    const unsigned char *act = masked ? L.active : nullptr;
    auto go = [&](auto rb) -> hipError_t {
        constexpr int RB = decltype(rb)::value;
        if (nd == 1)
            k_batch_matvec<1, RB><<<L.nmtiles, 256, 0, st>>>(L.probs, L.mtiles, L.nmtiles, act, x,
                                                             y, bsub, scheme, transpose, Vd, part,
                                                             ldp);
        else if (nd == 2)
            k_batch_matvec<2, RB><<<L.nmtiles, 256, 0, st>>>(L.probs, L.mtiles, L.nmtiles, act, x,
                                                             y, bsub, scheme, transpose, Vd, part,
                                                             ldp);
        else if (nd == 3)
            k_batch_matvec<3, RB><<<L.nmtiles, 256, 0, st>>>(L.probs, L.mtiles, L.nmtiles, act, x,
                                                             y, bsub, scheme, transpose, Vd, part,
                                                             ldp);
        else if (nd == 4)
            k_batch_matvec<4, RB><<<L.nmtiles, 256, 0, st>>>(L.probs, L.mtiles, L.nmtiles, act, x,
                                                             y, bsub, scheme, transpose, Vd, part,
                                                             ldp);
        else if (nd == -1)
            k_batch_matvec<-1, RB><<<L.nmtiles, 256, 0, st>>>(L.probs, L.mtiles, L.nmtiles, act, x,
                                                              y, bsub, scheme, transpose, nullptr,
                                                              part, ldp);
        else if (nd == 0)
            k_batch_matvec<0, RB><<<L.nmtiles, 256, 0, st>>>(L.probs, L.mtiles, L.nmtiles, act, x,
                                                             y, bsub, scheme, transpose, nullptr,
                                                             nullptr, 0);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    };
    switch (L.mrows) {
    case 2: return go(std::integral_constant<int, 2>{});
    case 4: return go(std::integral_constant<int, 4>{});
    case 8: return go(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t cgs_b(const BatchLaunch &L, const double *const *V, int nv, const double *w,
                        const double *coef, int cst, double *out, double *part, int ldp,
                        bool masked, hipStream_t st, const double *coef2 = nullptr)
{
    const unsigned char *act = masked ? L.active : nullptr;
#define AAO_BNV(K)                                                                          \
    if (nv <= K) {                                                                          \
        k_batch_cgs<MODE, K><<<L.nslabs, 256, 0, st>>>(L.probs, L.slabs, L.nslabs, act, V, nv, w, \
                                                      coef, cst, out, part, ldp, coef2);    \
        return hipGetLastError();                                                           \
    }
    AAO_BNV(1) AAO_BNV(4) AAO_BNV(8) AAO_BNV(16) AAO_BNV(32) AAO_BNV(64)
#undef AAO_BNV
    return hipErrorInvalidValue;
}

hipError_t batch_cgs(int mode, const BatchLaunch &L, const double *const *V, int nv, const double *w,
                     const double *coef, int cst, double *out, double *part, int ldp, bool masked,
                     hipStream_t st)
{
    if (mode == 0) return cgs_b<0>(L, V, nv, w, coef, cst, out, part, ldp, masked, st);
    if (mode == 1) return cgs_b<1>(L, V, nv, w, coef, cst, out, part, ldp, masked, st);
    return cgs_b<2>(L, V, nv, w, coef, cst, out, part, ldp, masked, st);
}

hipError_t batch_cgs_delayed(const BatchLaunch &L, const double *const *V, int nv,
                             const double *w, const BState &s, double *out, double *part, int ldp,
                             hipStream_t st)
{
    return cgs_b<3>(L, V, nv, w, s.coef, s.sst, out, part, ldp, true, st, s.h1);
}

hipError_t batch_reduce(const BatchLaunch &L, const double *part, int ldp, int cnt, double *sums,
                        int sst, bool masked, hipStream_t st, const int2 *ranges)
{
    if (cnt < 1) return hipSuccess;
    k_batch_reduce<<<dim3(L.count, cnt), 64, 0, st>>>(ranges ? ranges : L.pslabs, L.count,
                                                      masked ? L.active : nullptr, part, ldp, cnt,
                                                      sums, sst);
    return hipGetLastError();
}

hipError_t batch_small(int mode, int count, int j, int m, double tol, const BState &s,
                       hipStream_t st)
{
    k_batch_small<0><<<(count + 63) / 64, 64, 0, st>>>(mode, count, j, m, tol, s);
    return hipGetLastError();
}

hipError_t batch_backsolve(int count, int m, const BState &s, hipStream_t st)
{
    k_batch_backsolve<<<(count + 63) / 64, 64, 0, st>>>(count, m, s);
    return hipGetLastError();
}

hipError_t batch_axpy(const BatchLaunch &L, const double *const *Z, const BState &s, double *x,
                      bool overwrite, hipStream_t st, int kmax)
{
#define AAO_BAXPY(K)                                                                          \
    if (kmax <= K) {                                                                          \
        k_batch_axpy<K><<<L.nslabs, 256, 0, st>>>(L.probs, L.slabs, L.nslabs, Z, s, x,        \
                                                  overwrite ? 1 : 0);                         \
        return hipGetLastError();                                                             \
    }
    AAO_BAXPY(1) AAO_BAXPY(2) AAO_BAXPY(4) AAO_BAXPY(8) AAO_BAXPY(16) AAO_BAXPY(32) AAO_BAXPY(64)
#undef AAO_BAXPY
    return hipErrorInvalidValue;
}

hipError_t batch_count_active(const unsigned char *a, int count, int *nact, hipStream_t st)
{
    k_batch_copy_active<<<1, 64, 0, st>>>(a, count, nact);
    return hipGetLastError();
}

}  // namespace aao
