// Stencil and Krylov kernels: the block-Toeplitz matvec (arXiv 1810.00615,
// Sec. 2, eq. monolithicheat / C_BD2 / eq. nonuniformmonolithicheat), the
// right-hand side and initial data, and the classical Gram-Schmidt passes of the
// GMRES Arnoldi process.  All FP64, all memory-bound.
//
// Reductions are deterministic: every kernel writes one partial per workgroup
// (fixed in-block tree) into a value-major array part[i * ldp + block], and the
// partials are summed in a fixed order (k_reduce_parts, k_reduce_small).  No
// floating-point atomics.
#include "../../include/aao.h"
#include "aao_internal.h"
#include "lanes.h"

namespace aao {

constexpr int kRedThreads = 256;

// ------------------------------------------------------------ block reduce
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], int nv, double *part,
                                                   int ldp, double *red)
{
    // wave-level butterfly, then one value per wave through LDS
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < nv) {
            double v = acc[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) red[i * 16 + wv] = v;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[i * 16 + w];
        part[(size_t)i * ldp + blockIdx.x] = s;
    }
}

// Reduction kernels: one workgroup per 1024 elements, at most 16384 workgroups,
// grid-stride (measured on the GPU with a working set larger than the last-level
// cache: two vectors read at 5.9 TB/s, read-read-write at 5.3-5.4 TB/s, against
// 5.7 and 4.9 TB/s with 4096 workgroups).
int dot_blocks(size_t N)
{
    const size_t nb = (N + 1023) / 1024;
    return (int)(nb < 16384 ? (nb < 1 ? 1 : nb) : 16384);
}

// Grid-stride walk: element e0 + u * stride for u < U, stride = all threads.
struct Walk {
    size_t first, stride, end;
};
static __device__ __forceinline__ Walk grid_walk(size_t N)
{
    return {(size_t)blockIdx.x * blockDim.x + threadIdx.x, (size_t)gridDim.x * blockDim.x, N};
}

// ------------------------------------------------------------- CGS passes
// MODE 0: acc_i = sum_e V_i[e] w[e]
// MODE 1: w' = w - sum_i V_i c1_i;  acc_i = sum_e V_i[e] w'[e]
// MODE 2: w'' = w - sum_i V_i c1_i; out = w'' ; acc_0 = sum w''^2
template <int MODE, int NV>
__global__ void __launch_bounds__(kRedThreads)
k_cgs(VecList V, int nv, const double *__restrict__ w, const double *__restrict__ c1, size_t N,
      double *__restrict__ part, int ldp, double *__restrict__ out)
{
    __shared__ double red[NV * 16];
    double acc[NV];
    double cf[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) cf[i] = (MODE > 0 && i < nv) ? c1[i] : 0.0;
    // this block's slice, U elements per thread and iteration, all loads issued first
    constexpr int U = NV <= 4 ? 4 : (NV <= 8 ? 2 : 1);
    const Walk g = grid_walk(N);
    for (size_t e0 = g.first; e0 < g.end; e0 += (size_t)U * g.stride) {
        double we[U];
        double vv[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t e = e0 + (size_t)u * g.stride;
            const bool in = e < g.end;
            we[u] = in ? w[e] : 0.0;
#pragma unroll
            for (int i = 0; i < NV; ++i) vv[u][i] = (in && i < nv) ? V.p[i][e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t e = e0 + (size_t)u * g.stride;
            if (MODE == 0) {
#pragma unroll
                for (int i = 0; i < NV; ++i) acc[i] += vv[u][i] * we[u];
            } else {
                double s = we[u];
#pragma unroll
                for (int i = 0; i < NV; ++i) s -= vv[u][i] * cf[i];
                if (MODE == 1) {
#pragma unroll
                    for (int i = 0; i < NV; ++i) acc[i] += vv[u][i] * s;
                } else {
                    if (e < g.end) out[e] = s;
                    acc[0] += s * s;
                }
            }
        }
    }
    block_reduce_store<NV>(acc, MODE == 2 ? 1 : nv, part, ldp, red);
}

template <int MODE>
static hipError_t cgs_disp(const VecList &V, int nv, const double *w, const double *c1,
                           size_t N, double *part, int ldp, double *out, hipStream_t st)
{
    const int nb = dot_blocks(N);
#define AAO_NV(K)                                                                        \
    if (nv <= K) {                                                                       \
        k_cgs<MODE, K><<<nb, kRedThreads, 0, st>>>(V, nv, w, c1, N, part, ldp, out);     \
        return hipGetLastError();                                                        \
    }
    AAO_NV(1) AAO_NV(2) AAO_NV(3) AAO_NV(4) AAO_NV(8) AAO_NV(16) AAO_NV(32) AAO_NV(64)
#undef AAO_NV
    return hipErrorInvalidValue;
}

hipError_t launch_multidot(const VecList &V, int nv, const double *w, size_t N, double *part,
                           int ldp, hipStream_t st)
{
    return cgs_disp<0>(V, nv, w, nullptr, N, part, ldp, nullptr, st);
}

hipError_t launch_update_dot(const VecList &V, int nv, const double *w, const double *h,
                             size_t N, double *part, int ldp, hipStream_t st)
{
    return cgs_disp<1>(V, nv, w, h, N, part, ldp, nullptr, st);
}

hipError_t launch_update_norm(const VecList &V, int nv, const double *w, const double *h,
                              double *out, size_t N, double *part, int ldp, hipStream_t st)
{
    return cgs_disp<2>(V, nv, w, h, N, part, ldp, out, st);
}

// ------------------------------------ Arnoldi update, delayed re-orthogonalisation
// One pass over the basis of step j (S_0..S_j, S_j the pending vector p_j whose
// re-orthogonalisation was deferred to this step) and w = A z_j: forms the final
// v_j = sum_i cv_i S_i and the once-projected w1 = w - sum_i cw_i S_i, and the
// partials of S_i . w1 (i < j), v_j . w1 (value j) and w1 . w1 (value nv), from
// which the next step takes its re-orthogonalisation coefficients and w1's norm.
// vout may be S_j itself (each element is read before it is written, by the same
// thread); vout == nullptr when v_j = S_j needs no rewrite (j = 0).
template <int NV>
__global__ void __launch_bounds__(kRedThreads)
k_arnoldi_update(VecList S, int nv, const double *__restrict__ w, const double *__restrict__ cv,
                 const double *__restrict__ cw, double *vout, double *__restrict__ wout,
                 size_t N, double *__restrict__ part, int ldp)
{
    __shared__ double red[(NV + 1) * 16];
    double acc[NV + 1];
    double fv[NV], fw[NV];
    const int j = nv - 1;
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        fv[i] = i < nv ? cv[i] : 0.0;
        fw[i] = i < nv ? cw[i] : 0.0;
    }
    double nrm = 0.0;
    constexpr int U = NV <= 4 ? 4 : (NV <= 8 ? 2 : 1);
    const Walk g = grid_walk(N);
    for (size_t e0 = g.first; e0 < g.end; e0 += (size_t)U * g.stride) {
        double we[U];
        double vv[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t e = e0 + (size_t)u * g.stride;
            const bool in = e < g.end;
            we[u] = in ? w[e] : 0.0;
#pragma unroll
            for (int i = 0; i < NV; ++i) vv[u][i] = (in && i < nv) ? S.p[i][e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t e = e0 + (size_t)u * g.stride;
            double vj = 0.0, s = we[u];
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                vj += fv[i] * vv[u][i];
                s -= fw[i] * vv[u][i];
            }
            if (e < g.end) {
                if (vout) vout[e] = vj;
                wout[e] = s;
            }
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] += (i == j ? vj : vv[u][i]) * s;
            nrm += s * s;
        }
    }
#pragma unroll
    for (int i = 0; i <= NV; ++i)
        if (i == nv) acc[i] = nrm;
    block_reduce_store<NV + 1>(acc, nv + 1, part, ldp, red);
}

hipError_t launch_arnoldi_update(const VecList &S, int nv, const double *w, const double *cv,
                                 const double *cw, double *vout, double *wout, size_t N,
                                 double *part, int ldp, hipStream_t st)
{
    const int nb = dot_blocks(N);
#define AAO_NV(K)                                                                          \
    if (nv <= K) {                                                                         \
        k_arnoldi_update<K><<<nb, kRedThreads, 0, st>>>(S, nv, w, cv, cw, vout, wout, N,   \
                                                          part, ldp);                      \
        return hipGetLastError();                                                          \
    }
    AAO_NV(1) AAO_NV(2) AAO_NV(3) AAO_NV(4) AAO_NV(8) AAO_NV(16) AAO_NV(32) AAO_NV(63)
#undef AAO_NV
    return hipErrorInvalidValue;
}

// Fixed-order sum of the per-block partials: sums[i] = sum_b part[i*ldp + b].
__global__ void __launch_bounds__(256)
k_reduce_parts(const double *__restrict__ part, int nblk, int ldp, double *__restrict__ sums)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    const double *p = part + (size_t)i * ldp;
    double s = 0.0;
    // sixteen loads in flight per thread, then added in a fixed order
    for (int base = 0; base < nblk; base += 16 * (int)blockDim.x) {
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int b = base + k * (int)blockDim.x + (int)threadIdx.x;
            v[k] = b < nblk ? p[b] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) s += v[k];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[i] = red[0];
}

hipError_t launch_reduce_parts(const double *part, int nblk, int ldp, int cnt, double *sums,
                               hipStream_t st)
{
    k_reduce_parts<<<cnt, 256, 0, st>>>(part, nblk, ldp, sums);
    return hipGetLastError();
}

// ------------------------------------------------------- small vector ops
// x = (accumulate ? x : 0) + sum_i Z_i y_i; NZ >= nz, all loads of an iteration
// issued before the sums
template <int NZ>
__global__ void __launch_bounds__(kRedThreads)
k_multi_axpy(VecList Z, int nz, CoefList y, double *__restrict__ x, size_t N, int accumulate)
{
    constexpr int U = NZ <= 2 ? 4 : (NZ <= 8 ? 2 : 1);
    double yc[NZ];
#pragma unroll
    for (int i = 0; i < NZ; ++i) yc[i] = i < nz ? y.v[i] : 0.0;
    const Walk g = grid_walk(N);
    for (size_t e0 = g.first; e0 < g.end; e0 += (size_t)U * g.stride) {
        double s[U];
        double zz[U][NZ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t e = e0 + (size_t)u * g.stride;
            const bool in = e < g.end;
            s[u] = (accumulate && in) ? x[e] : 0.0;
#pragma unroll
            for (int i = 0; i < NZ; ++i) zz[u][i] = (in && i < nz) ? Z.p[i][e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t e = e0 + (size_t)u * g.stride;
#pragma unroll
            for (int i = 0; i < NZ; ++i) s[u] += zz[u][i] * yc[i];
            if (e < g.end) x[e] = s[u];
        }
    }
}

static int grid_for(size_t N)
{
    size_t g = (N + 255) / 256;
    return (int)(g < 16384 ? (g < 1 ? 1 : g) : 16384);
}

hipError_t launch_multi_axpy(const VecList &Z, int nz, const CoefList &y, double *x, size_t N,
                             bool accumulate, hipStream_t st)
{
    const int nb = dot_blocks(N);
#define AAO_NZ(K)                                                                          \
    if (nz <= K) {                                                                         \
        k_multi_axpy<K><<<nb, kRedThreads, 0, st>>>(Z, nz, y, x, N, accumulate ? 1 : 0);   \
        return hipGetLastError();                                                          \
    }
    AAO_NZ(1) AAO_NZ(2) AAO_NZ(3) AAO_NZ(4) AAO_NZ(8) AAO_NZ(16) AAO_NZ(32) AAO_NZ(64)
#undef AAO_NZ
    return hipErrorInvalidValue;
}

__global__ void k_scale(const double *__restrict__ w, const double *__restrict__ sc, double a,
                        double *__restrict__ out, size_t N)
{
    const double f = sc ? *sc : a;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride)
        out[e] = w[e] * f;
}

hipError_t launch_scale(const double *w, const double *scale, double *out, size_t N,
                        hipStream_t st)
{
    k_scale<<<grid_for(N), 256, 0, st>>>(w, scale, 0.0, out, N);
    return hipGetLastError();
}

hipError_t launch_scale_h(const double *w, double a, double *out, size_t N, hipStream_t st)
{
    k_scale<<<grid_for(N), 256, 0, st>>>(w, nullptr, a, out, N);
    return hipGetLastError();
}

__global__ void k_fill(double *x, double v, size_t N)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) x[e] = v;
}

hipError_t launch_fill(double *x, double v, size_t N, hipStream_t st)
{
    k_fill<<<grid_for(N), 256, 0, st>>>(x, v, N);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kRedThreads)
k_dot1(const double *__restrict__ a, const double *__restrict__ b, size_t N,
       double *__restrict__ part)
{
    __shared__ double red[2 * 16];
    double acc[1] = {0.0};
    constexpr int U = 4;
    const Walk g = grid_walk(N);
    for (size_t e0 = g.first; e0 < g.end; e0 += (size_t)U * g.stride) {
        double av[U], bv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t e = e0 + (size_t)u * g.stride;
            av[u] = e < g.end ? a[e] : 0.0;
            bv[u] = e < g.end ? b[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc[0] += av[u] * bv[u];
    }
    block_reduce_store<1>(acc, 1, part, 1, red);
}

hipError_t launch_dot1_parts(const double *a, const double *b, size_t N, double *part,
                             hipStream_t st)
{
    k_dot1<<<dot_blocks(N), kRedThreads, 0, st>>>(a, b, N, part);
    return hipGetLastError();
}

// -------------------------------------------------------- matvec (Sec. 2)
// y_k = sum_{m=0}^{s} (a_m M + b_m^{(k)} kappa K) x_{k-m}   (x_{k+m} if transposed)
// with b_0^{(k)} = tau_k when variable steps are given.  y = bsub - A x if bsub.
//
// Each thread owns one spatial column and R consecutive output time levels; the
// R + S input rows it needs (S = scheme order) are all loaded before any output
// is formed, one aligned load per row, so the loads of a lane are in flight
// together.  The i -+ 1 neighbours come from the adjacent lanes by a cross-lane
// move (DPP wave shift when DPP is set, else ds_bpermute); lanes 0 and 63 fetch
// the neighbour outside their wave with a second, two-lane load.  With nv > 0 the
// kernel also leaves the block partials of V_q . y, q < nv (value-major, block id
// y * gridDim.x + x): the first Gram-Schmidt pass, or with nv = 1 and V_0 = y the
// squared norm of a residual (from registers).
// DOTS: 0 none, 1 partials of V_q . y (q < nv), 2 the partial of y . y only
template <int S, int R, bool DPP, int DOTS, int NZ = 0>
__global__ void __launch_bounds__(256)
k_matvec(const double *__restrict__ x, double *__restrict__ y, const double *__restrict__ bsub,
         int n, int ell, Scheme sc, double kappa, const double *__restrict__ tau_k, int transpose,
         VecList V, int nv, double *__restrict__ part, int ldp, MatvecComb cb = {})
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool col = i < n;          // lanes past n still take part in the lane moves
    const double h = 1.0 / (n + 1.0);
    const int k0 = blockIdx.y * R;
    const int k1 = min(k0 + R, ell);                // output rows [k0, k1)
    const int nin = (k1 - k0) + S;                  // input rows touched by the block
    constexpr int NR = R + S;
    const int je = lane == 0 ? i - 1 : i + 1;       // outside neighbour of lanes 0 / 63
    const bool edge = (lane == 0 || lane == 63) && je >= 0 && je < n;
    double c[NR], e[NR];
#pragma unroll
    for (int it = 0; it < NR; ++it) {
        const int kk = transpose ? (k1 - 1 + S - it) : (k0 - S + it);
        const bool in = it < nin && kk >= 0 && kk < ell;
        if (NZ == 0) {
            const double *row = x + (size_t)(in ? kk : 0) * n;
            c[it] = (in && col) ? row[i] : 0.0;
            e[it] = (in && edge) ? row[je] : 0.0;
        } else {
            // x = sum_q c_q Z_q formed on the fly (and stored for the owned rows below)
            double cc = 0.0, ee = 0.0;
#pragma unroll
            for (int q = 0; q < NZ; ++q) {
                const double *row = cb.z[q] + (size_t)(in ? kk : 0) * n;
                cc += cb.c[q] * ((in && col) ? row[i] : 0.0);
                ee += cb.c[q] * ((in && edge) ? row[je] : 0.0);
            }
            c[it] = cc;
            e[it] = ee;
        }
    }
    // the rows of bsub and of the first two basis vectors are loaded with x, so that
    // their latency overlaps the x loads instead of following the stencil
    double bs[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int k = transpose ? (k1 - 1 - r) : (k0 + r);
        bs[r] = (bsub && col && r < nin - S) ? bsub[(size_t)k * n + i] : 0.0;
    }
    constexpr int G = 2;
    double vq0[G][R];
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = transpose ? (k1 - 1 - r) : (k0 + r);
            vq0[u][r] = (DOTS == 1 && u < nv && col && r < nin - S) ? V.p[u][(size_t)k * n + i]
                                                                     : 0.0;
        }
    // l, c, r of the last S+1 input rows; the time combination is formed before
    // the space stencil, so that cancelling time differences (BD2: x_k - 2 x_{k-1}
    // + x_{k-2}) are taken on the raw values
    double wl[S + 1] = {}, wc[S + 1] = {}, wr[S + 1] = {};
    double yv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) yv[r] = 0.0;
#pragma unroll
    for (int it = 0; it < NR; ++it) {
        double l = lane_from_left<DPP>(c[it]);
        double r = lane_from_right<DPP>(c[it]);
        if (lane == 0) l = e[it];
        if (lane == 63) r = e[it];
#pragma unroll
        for (int m = S; m > 0; --m) {
            wl[m] = wl[m - 1];
            wc[m] = wc[m - 1];
            wr[m] = wr[m - 1];
        }
        wl[0] = l;
        wc[0] = c[it];
        wr[0] = r;
        if (it < S || it >= nin) continue;
        // output row k uses input rows k -+ m, m = 0..S
        const int k = transpose ? (k1 - 1 + S - it) : (k0 - S + it);
        double al = 0.0, ac = 0.0, ar = 0.0, bl = 0.0, bc = 0.0, br = 0.0;
#pragma unroll
        for (int m = 0; m <= S; ++m) {
            const double am = sc.a[m];
            double bm = sc.b[m];
            if (m == 0 && tau_k) bm = tau_k[k];
            bm *= kappa;
            al += am * wl[m];
            ac += am * wc[m];
            ar += am * wr[m];
            bl += bm * wl[m];
            bc += bm * wc[m];
            br += bm * wr[m];
        }
        const double v = (h / 6.0) * (al + 4.0 * ac + ar) + (1.0 / h) * (2.0 * bc - bl - br);
        const double out = bsub ? bs[it - S] - v : v;
        yv[it - S] = out;
        if (col && y) y[(size_t)k * n + i] = out;
        if (NZ > 0 && col) cb.xout[(size_t)k * n + i] = c[it];   // the owned rows of x
    }
    if (DOTS == 0) return;
    __shared__ double red[kMaxVecs * 4];
    const int wv = threadIdx.x >> 6;
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    if (DOTS == 2) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) acc += (col && r < nin - S) ? yv[r] * yv[r] : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) red[wv] = acc;
        __syncthreads();
        if (threadIdx.x == 0) part[blk] = ((red[0] + red[1]) + red[2]) + red[3];
        return;
    }
    // partial dot products V_q . y over this block's tile (first Gram-Schmidt pass)
    // two basis vectors at a time, all their loads issued before the sums (the first
    // two with x)
    for (int q0 = 0; q0 < nv; q0 += G) {
        double acc[G];
        double vq[G][R];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            acc[u] = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = transpose ? (k1 - 1 - r) : (k0 + r);
                vq[u][r] = q0 == 0 ? vq0[u][r]
                                   : (q0 + u < nv && col && r < nin - S)
                                         ? V.p[q0 + u][(size_t)k * n + i]
                                         : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
#pragma unroll
            for (int r = 0; r < R; ++r) acc[u] += vq[u][r] * yv[r];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc[u] += __shfl_down(acc[u], off, 64);
            if (lane == 0 && q0 + u < nv) red[(q0 + u) * 4 + wv] = acc[u];
        }
    }
    {
        // y . y as value nv (the Pythagorean estimate of the projected norm)
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) acc += (col && r < nin - S) ? yv[r] * yv[r] : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) red[nv * 4 + wv] = acc;
    }
    __syncthreads();
    for (int q = threadIdx.x; q <= nv; q += blockDim.x)
        part[(size_t)q * ldp + blk] = ((red[q * 4] + red[q * 4 + 1]) + red[q * 4 + 2]) + red[q * 4 + 3];
}

// Launch shapes: code = 3 v + r, R = 4 << r rows per thread, v = 1 for DPP lane
// moves, v = 0 for ds_bpermute.
int matvec_num_configs() { return 6; }
int matvec_default_config() { return 3 + 2; }

template <int S>
static hipError_t matvec_disp(int cfg, const double *x, double *y, const double *bsub, int n,
                              int ell, Scheme sc, double kappa, const double *tau_k,
                              int transpose, const VecList &V, int nv, double *part, int ldp,
                              hipStream_t st)
{
    const int R = 4 << (cfg % 3);
    dim3 grid((n + 255) / 256, (ell + R - 1) / R);
#define AAO_MV(C, RR, D)                                                                    \
    case C:                                                                                 \
        if (nv > 0 && V.p[0] == y)                                                         \
            k_matvec<S, RR, D, 2><<<grid, 256, 0, st>>>(x, y, bsub, n, ell, sc, kappa, tau_k, \
                                                        transpose, V, 1, part, ldp);          \
        else if (nv > 0)                                                                    \
            k_matvec<S, RR, D, 1><<<grid, 256, 0, st>>>(x, y, bsub, n, ell, sc, kappa, tau_k, \
                                                        transpose, V, nv, part, ldp);         \
        else                                                                                \
            k_matvec<S, RR, D, 0><<<grid, 256, 0, st>>>(x, y, bsub, n, ell, sc, kappa, tau_k, \
                                                        transpose, V, 0, part, ldp);          \
        break;
    switch (cfg) {
        AAO_MV(0, 4, false)
        AAO_MV(1, 8, false)
        AAO_MV(2, 16, false)
        AAO_MV(3, 4, true)
        AAO_MV(4, 8, true)
        AAO_MV(5, 16, true)
    default: return hipErrorInvalidValue;
    }
#undef AAO_MV
    return hipGetLastError();
}

// Residual check of x = sum_q c_q Z_q (nz <= 4, DPP launch shapes only): x is formed
// on the fly, stored, and the launch writes the partials of |bsub - A x|^2.
template <int S>
static hipError_t matvec_comb_disp(int cfg, const MatvecComb &cb, int nz, const double *bsub,
                                   int n, int ell, Scheme sc, double kappa, const double *tau_k,
                                   int transpose, double *part, hipStream_t st)
{
    const int R = 4 << (cfg % 3);
    dim3 grid((n + 255) / 256, (ell + R - 1) / R);
    const VecList none{};
#define AAO_MC(RR, K)                                                                           \
    if (R == RR && nz == K) {                                                                   \
        k_matvec<S, RR, true, 2, K><<<grid, 256, 0, st>>>(nullptr, nullptr, bsub, n, ell, sc,   \
                                                          kappa, tau_k, transpose, none, 1,     \
                                                          part, 0, cb);                         \
        return hipGetLastError();                                                               \
    }
    AAO_MC(4, 1) AAO_MC(4, 2) AAO_MC(4, 3) AAO_MC(4, 4)
    AAO_MC(8, 1) AAO_MC(8, 2) AAO_MC(8, 3) AAO_MC(8, 4)
    AAO_MC(16, 1) AAO_MC(16, 2) AAO_MC(16, 3) AAO_MC(16, 4)
#undef AAO_MC
    return hipErrorInvalidValue;
}

bool matvec_comb_ok(int cfg, int nz)
{
    if (cfg < 0 || cfg >= matvec_num_configs()) cfg = matvec_default_config();
    return cfg >= 3 && nz >= 1 && nz <= 4;
}

hipError_t launch_matvec_comb(const MatvecComb &cb, int nz, const double *bsub, int n, int ell,
                              Scheme sc, double kappa, const double *tau_k, int transpose,
                              hipStream_t st, int cfg, double *part, int ldp)
{
    if (cfg < 0 || cfg >= matvec_num_configs()) cfg = matvec_default_config();
    if (!matvec_comb_ok(cfg, nz) || !part || !cb.xout || matvec_blocks(n, ell, cfg) > ldp)
        return hipErrorInvalidValue;
    switch (sc.s) {
    case 1:
        return matvec_comb_disp<1>(cfg, cb, nz, bsub, n, ell, sc, kappa, tau_k, transpose, part, st);
    case 2:
        return matvec_comb_disp<2>(cfg, cb, nz, bsub, n, ell, sc, kappa, tau_k, transpose, part, st);
    case 3:
        return matvec_comb_disp<3>(cfg, cb, nz, bsub, n, ell, sc, kappa, tau_k, transpose, part, st);
    default: return hipErrorInvalidValue;
    }
}

int matvec_blocks(int n, int ell, int cfg)
{
    if (cfg < 0 || cfg >= matvec_num_configs()) cfg = matvec_default_config();
    const int R = 4 << (cfg % 3);
    return ((n + 255) / 256) * ((ell + R - 1) / R);
}

// out = s r - E z, E = blockdiag(sigma_k kappa K) (the residual a Neumann term of
// eq. preconapprox1 transforms), s = *scale or 1; kap_h = kappa / h.
__global__ void k_neumann_rhs(const double *__restrict__ r, const double *__restrict__ scale,
                              const double *__restrict__ z, const double *__restrict__ sigk,
                              double kap_h, int n, int ell, double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= n) return;
    const size_t o = (size_t)k * n + i;
    const double zl = i > 0 ? z[o - 1] : 0.0, zr = i < n - 1 ? z[o + 1] : 0.0;
    const double s = scale ? *scale : 1.0;
    out[o] = s * r[o] - sigk[k] * kap_h * (2.0 * z[o] - zl - zr);
}

hipError_t launch_neumann_rhs(const double *r, const double *scale, const double *z,
                              const double *sigk, double kappa, int n, int ell, double *out,
                              hipStream_t st)
{
    dim3 grid((n + 255) / 256, ell);
    k_neumann_rhs<<<grid, 256, 0, st>>>(r, scale, z, sigk, kappa * (n + 1.0), n, ell, out);
    return hipGetLastError();
}

// Matvec of the schemes with start-up rows (BD4) or a block above the diagonal
// (central differences): y_k = sum_m A_{k,k-m} x_{k-m}, or (transpose) y_k =
// sum_m A_{k+m,k} x_{k+m} (every block symmetric); y = bsub - A x if bsub.  A thread
// owns one spatial node and kMvWalkSeg consecutive output levels (downwards in time
// for the transpose); the kMvWalkSeg + W - 1 input levels they touch (W = s + up + 1)
// are loaded first, all at once (clamped, masked), and reduced to M x and K x at the
// node, so each input level is read once per segment.  Slot j holds level
// k0 - dir (s - j); output t takes offset m = c - up from slot t + W - 1 - c.  The
// blocks come from scheme_block (start-up rows, the block above the diagonal).
constexpr int kMvWalkSeg = 8;

template <int W>
__global__ void __launch_bounds__(256)
k_matvec_walk(const double *__restrict__ x, double *__restrict__ y,
              const double *__restrict__ bsub, int n, int ell, Scheme sc, double kappa,
              int transpose)
{
    constexpr int NL = kMvWalkSeg + W - 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int up = sc.up;
    const int dir = transpose ? -1 : 1;
    const int kb = blockIdx.y * kMvWalkSeg;
    const int ke = min(ell, kb + kMvWalkSeg);
    const int k0 = transpose ? ke - 1 : kb;
    const int cnt = ke - kb;
    const double h = 1.0 / (n + 1.0);
    const int il = i > 0 ? i - 1 : 0, ir = i < n - 1 ? i + 1 : i;
    const double ml = i > 0 ? 1.0 : 0.0, mr = i < n - 1 ? 1.0 : 0.0;
    double P[NL], Q[NL];               // (M x)_i and (K x)_i of the touched levels
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const int L = k0 - dir * (sc.s - j);
        const double w = (L >= 0 && L < ell) ? 1.0 : 0.0;
        const double *row = x + (size_t)(L >= 0 && L < ell ? L : 0) * n;
        const double l = w * ml * row[il], cc = w * row[i], r = w * mr * row[ir];
        P[j] = (h / 6.0) * (l + 4.0 * cc + r);
        Q[j] = (1.0 / h) * (2.0 * cc - l - r);
    }
#pragma unroll
    for (int t = 0; t < kMvWalkSeg; ++t) {
        if (t >= cnt) continue;
        const int k = k0 + dir * t;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const int m = c - up;
            const int src = transpose ? k + m : k - m;
            const int row = transpose ? src : k;
            double cm, cb;
            if (src >= 0 && src < ell && scheme_block(sc, row, m, cm, cb))
                acc += cm * P[t + W - 1 - c] + cb * kappa * Q[t + W - 1 - c];
        }
        const size_t o = (size_t)k * n + i;
        y[o] = bsub ? bsub[o] - acc : acc;
    }
}

hipError_t launch_matvec(const double *x, double *y, const double *bsub, int n, int ell,
                         Scheme sc, double kappa, const double *tau_k, int transpose,
                         hipStream_t st, int cfg, const VecList *V, int nv, double *part, int ldp)
{
    if (scheme_generic(sc)) {
        // no fused dot products, no variable steps for these schemes
        if (nv > 0 || tau_k || !y) return hipErrorInvalidValue;
        dim3 grid((n + 255) / 256, (ell + kMvWalkSeg - 1) / kMvWalkSeg);
        switch (sc.s + sc.up + 1) {
        case 2: k_matvec_walk<2><<<grid, 256, 0, st>>>(x, y, bsub, n, ell, sc, kappa, transpose); break;
        case 3: k_matvec_walk<3><<<grid, 256, 0, st>>>(x, y, bsub, n, ell, sc, kappa, transpose); break;
        case 4: k_matvec_walk<4><<<grid, 256, 0, st>>>(x, y, bsub, n, ell, sc, kappa, transpose); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (cfg < 0 || cfg >= matvec_num_configs()) cfg = matvec_default_config();
    if (nv > 0 && (!V || !part || nv >= kMaxVecs || matvec_blocks(n, ell, cfg) > ldp))
        return hipErrorInvalidValue;
    static const VecList none{};
    const VecList &L = V ? *V : none;
    switch (sc.s) {
    case 1:
        return matvec_disp<1>(cfg, x, y, bsub, n, ell, sc, kappa, tau_k, transpose, L, nv, part,
                              ldp, st);
    case 2:
        return matvec_disp<2>(cfg, x, y, bsub, n, ell, sc, kappa, tau_k, transpose, L, nv, part,
                              ldp, st);
    case 3:
        return matvec_disp<3>(cfg, x, y, bsub, n, ell, sc, kappa, tau_k, transpose, L, nv, part,
                              ldp, st);
    default: return hipErrorInvalidValue;
    }
}

// y = (cm M + ck K) x (+ (cm2 M + ck2 K) x2 + (cm3 M + ck3 K) x3), one n-vector
__global__ void k_mk(const double *__restrict__ x, double cm, double ck,
                     const double *__restrict__ x2, double cm2, double ck2,
                     const double *__restrict__ x3, double cm3, double ck3,
                     double *__restrict__ y, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h = 1.0 / (n + 1.0);
    auto term = [&](const double *z, double a, double c) {
        const double zl = i > 0 ? z[i - 1] : 0.0, zr = i < n - 1 ? z[i + 1] : 0.0;
        return a * (h / 6.0) * (zl + 4.0 * z[i] + zr) + c * (1.0 / h) * (2.0 * z[i] - zl - zr);
    };
    double v = term(x, cm, ck);
    if (x2) v += term(x2, cm2, ck2);
    if (x3) v += term(x3, cm3, ck3);
    y[i] = v;
}

hipError_t launch_mk(const double *x, double cm, double ck, const double *x2, double cm2,
                     double ck2, double *y, int n, hipStream_t st, const double *x3, double cm3,
                     double ck3)
{
    k_mk<<<(n + 255) / 256, 256, 0, st>>>(x, cm, ck, x2, cm2, ck2, x3, cm3, ck3, y, n);
    return hipGetLastError();
}

// ------------------------------------------------ initial data and rhs
// u0_i = sum_m amps_m (g_m / mu_m) sin(q_m pi x_i): the L2 projection of a sine
// series (each sine mode is an eigenvector of M with eigenvalue
// mu = (h/3)(2 + cos q pi h); its exact load vector is g sin(q pi x_i),
// g = 4 sin^2(q pi h / 2) / (h q^2 pi^2)).
__global__ void k_project_sine(double *__restrict__ u0, int n, int J,
                               const int *__restrict__ modes, const double *__restrict__ amps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h = 1.0 / (n + 1.0);
    const long long period = 2LL * (n + 1);
    double s = 0.0;
    for (int m = 0; m < J; ++m) {
        const long long q = modes[m];
        const double sh = sinpi(0.5 * (double)q / (double)(n + 1));
        const double g = 4.0 * sh * sh / (h * (double)q * (double)q * M_PI * M_PI);
        const double mu = (h / 3.0) * (2.0 + cospi((double)q / (double)(n + 1)));
        const long long arg = (q * (long long)(i + 1)) % period;
        s += amps[m] * (g / mu) * sinpi((double)arg / (double)(n + 1));
    }
    u0[i] = s;
}

hipError_t launch_project_sine(double *u0, int n, int J, const int *modes, const double *amps,
                               hipStream_t st)
{
    k_project_sine<<<(n + 255) / 256, 256, 0, st>>>(u0, n, J, modes, amps);
    return hipGetLastError();
}

// Right-hand sides (the u0 / v0 terms of the first rows moved to the right):
//   heat: b_1 = M u0;
//   BD2:  b_1 = A_0 (u0 + tau v0), b_2 = -M u0;
//   BD4:  b_1 = B (u0 + tau v0), b_2 = -M u0, b_3 = M u0 (B = M + tau^2 kappa K);
//   CD:   b_1 = -M u0;
// other rows 0.  wave: BD2 / BD4 (start-up row with tau^2 kappa K: kb = tau^2 kappa).
__global__ void k_build_rhs(double *__restrict__ b, const double *__restrict__ u0,
                            const double *__restrict__ v0, int n, int ell, int id, double kb,
                            double tau)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= n) return;
    const double h = 1.0 / (n + 1.0);
    const bool wave = id == AAO_WAVE_BD2 || id == AAO_WAVE_BD4;
    const double ul = i > 0 ? u0[i - 1] : 0.0, ur = i < n - 1 ? u0[i + 1] : 0.0;
    const double mu = (h / 6.0) * (ul + 4.0 * u0[i] + ur);
    double v = 0.0;
    if (k == 0) {
        if (id == AAO_WAVE_CD) {
            v = -mu;
        } else {
            auto w = [&](int p) {
                if (p < 0 || p >= n) return 0.0;
                return u0[p] + (v0 ? tau * v0[p] : 0.0);
            };
            const double wl = w(i - 1), wc = w(i), wr = w(i + 1);
            v = (h / 6.0) * (wl + 4.0 * wc + wr);
            if (wave) v += kb * (1.0 / h) * (2.0 * wc - wl - wr);
        }
    } else if (k == 1 && wave) {
        v = -mu;
    } else if (k == 2 && id == AAO_WAVE_BD4) {
        v = mu;
    }
    b[(size_t)k * n + i] = v;
}

hipError_t launch_build_rhs(double *b, const double *u0, const double *v0, int n, int ell,
                            Scheme sc, double kappa, double tau, hipStream_t st)
{
    const bool wave = sc.id == AAO_WAVE_BD2 || sc.id == AAO_WAVE_BD4;
    dim3 grid((n + 255) / 256, ell);
    k_build_rhs<<<grid, 256, 0, st>>>(b, u0, wave ? v0 : nullptr, n, ell, sc.id,
                                      tau * tau * kappa, tau);
    return hipGetLastError();
}

// ----------------------------------------------------- gradient (kappa)
// partials of sum_k sum_m c_m^{(k)} lam_k . (K u_{k-m}),  c_m^{(k)} the K coefficient
// (without kappa) of block (k, k - m): b_m, tau_k for m = 0 with variable steps, the
// start-up rows' own, bu above the diagonal
__global__ void __launch_bounds__(kRedThreads)
k_grad_kappa(const double *__restrict__ U, const double *__restrict__ lam, int n, int ell,
             Scheme sc, const double *__restrict__ tau_k, double *__restrict__ part)
{
    __shared__ double red[2 * 16];
    double acc[1] = {0.0};
    const double hinv = n + 1.0;
    const size_t N = (size_t)n * ell;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += stride) {
        const int k = (int)(e / n);
        const int i = (int)(e - (size_t)k * n);
        double ku = 0.0;
        for (int m = -sc.up; m <= sc.s; ++m) {
            double am = 0.0, cm = 0.0;
            if (!scheme_block(sc, k, m, am, cm)) continue;
            if (m == 0 && tau_k) cm = tau_k[k];
            if (cm == 0.0 || k - m < 0 || k - m >= ell) continue;
            const double *ur = U + (size_t)(k - m) * n;
            const double ul = i > 0 ? ur[i - 1] : 0.0, urr = i < n - 1 ? ur[i + 1] : 0.0;
            ku += cm * hinv * (2.0 * ur[i] - ul - urr);
        }
        acc[0] += lam[e] * ku;
    }
    block_reduce_store<1>(acc, 1, part, 1, red);
}

hipError_t launch_grad_kappa_parts(const double *U, const double *lam, int n, int ell,
                                   Scheme sc, const double *tau_k, double *part, int nblk,
                                   hipStream_t st)
{
    k_grad_kappa<<<nblk, kRedThreads, 0, st>>>(U, lam, n, ell, sc, tau_k, part);
    return hipGetLastError();
}

}  // namespace aao

namespace aao {

// Fixed-order reduction of the partials of one Krylov step followed by its scalar
// update, in one block (16 waves; every thread sums a fixed strided subset of the
// partials of every value, each wave adds its threads' sums, then thread 0 adds the
// 16 wave sums in order).  The basis
// is stored unnormalised with scales vs (v_i = vs_i V_i), so that no host round
// trip sits between the Gram-Schmidt passes; d are the reduced raw dot products.
//   mode 0: h1_i = vs_i d_i, c_i = vs_i h1_i             (first projection, i < nv)
//   mode 1: h2_i = vs_i d_i, c_i += vs_i h2_i            (re-orthogonalisation)
//   mode 2: nrm = sqrt(d_0), vs_nv = 1/nrm, host[0..nv] = (h1 + h2, nrm)
//   mode 3: nrm = sqrt(d_0), vs_0 = 1/nrm, host[kHostBeta] = nrm    (restart vector)
//   mode 4: host[kHostBB] = d_0 (= b.b); with nv == 1 also vs_0 = 1/sqrt(d_0)
//           and host[kHostBeta] = sqrt(d_0)       (zero initial guess: V_0 = b)
//   mode 5: delayed re-orthogonalisation after the matvec of step j = nv - 1:
//           coefficients cv, cw of the update pass, host[0..j] = first projections,
//           host[kHostWW] = w . w (partials: S_i . w for i < nv, then w . w)
//   mode 6: after the update pass: vs_nv = 1/|w1|, a_i (next step's coefficients),
//           host[nv] = |w1|, host[kHostA + i] = a_i
// host: mapped pinned memory; host[kHostFail] receives the breakdown flag, and
// host[kHostSeq] the launch's sequence number once everything else is visible.
__global__ void __launch_bounds__(1024)
k_reduce_small(const double *__restrict__ part, int nblk, int ldp, SmallArgs a)
{
    __shared__ double wsum[16][kMaxVecs];
    __shared__ double sums[kMaxVecs + 1];   // final sums (LDS: indexed at run time)
    // the step's scalars, read once by parallel loads: the serial update below reads
    // them from LDS instead of one dependent global load after another
    __shared__ double lvs[kMaxVecs + 1], la[kMaxVecs + 1], lh1[kMaxVecs + 1],
        lh2[kMaxVecs + 1], lc[kMaxVecs + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int cnt = (a.mode <= 1) ? a.nv : (a.mode >= 5 ? a.nv + 1 : 1);
    const int nv = a.nv;
    if ((int)threadIdx.x <= nv) {
        const int i = threadIdx.x;
        lvs[i] = a.vs[i];
        if (a.mode >= 5) la[i] = a.a[i];
        if (a.mode == 1) lc[i] = a.c[i];
        if (a.mode == 2) {
            lh1[i] = a.h1[i];
            lh2[i] = a.h2[i];
        }
    }
    if (nblk == 1) {
        // one partial per value (pre-summed): value i is thread i's load
        if ((int)threadIdx.x < cnt) sums[threadIdx.x] = part[(size_t)threadIdx.x * ldp];
        __syncthreads();
    } else {
        // thread t sums the partials t, t + 1024, ... of every value, the loads of two
        // values (32 per thread) in flight at a time; then each wave and finally one
        // thread per value add in a fixed order
        for (int i0 = 0; i0 < cnt; i0 += 2) {
            double s[2] = {0.0, 0.0};
            for (int base = 0; base < nblk; base += 16 * 1024) {
                double v[2][16];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const double *p = part + (size_t)min(i0 + q, cnt - 1) * ldp;
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int b = base + k * 1024 + (int)threadIdx.x;
                        v[q][k] = (i0 + q < cnt && b < nblk) ? p[b] : 0.0;
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int k = 0; k < 16; ++k) s[q] += v[q][k];
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_down(s[q], off, 64);
                if (lane == 0 && i0 + q < cnt) wsum[wv][i0 + q] = s[q];
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            double s = 0.0;
            for (int w = 0; w < 16; ++w) s += wsum[w][threadIdx.x];
            sums[threadIdx.x] = s;
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (a.mode == 5) {
        // delayed re-orthogonalisation, after w = A z_j (sums: S_i . w, i <= j):
        // p_j = sum_{i<j} a_i v_i + alpha v_j with |p_j| = 1, so
        //   alpha = sqrt(1 - |a|^2),  v_j = (p_j - sum a_i v_i) / alpha,
        //   h_i = v_i . w = b_i (i < j),  h_j = v_j . w = (p_j . w - a . b) / alpha,
        //   w1 = w - sum_{i<j} h_i v_i - h_j v_j.
        const int j = nv - 1;
        double aa = 0.0, ab = 0.0;
        for (int i = 0; i < j; ++i) {
            const double bi = lvs[i] * sums[i];
            aa += la[i] * la[i];
            ab += la[i] * bi;
        }
        const double alpha = j > 0 ? sqrt(fmax(1.0 - aa, 1e-300)) : 1.0;
        const double hj = (lvs[j] * sums[j] - ab) / alpha;
        for (int i = 0; i < j; ++i) {
            const double bi = lvs[i] * sums[i];
            a.cv[i] = -la[i] * lvs[i] / alpha;
            a.cw[i] = (bi - la[i] * hj / alpha) * lvs[i];
            a.host[i] = bi;
        }
        a.cv[j] = lvs[j] / alpha;
        a.cw[j] = hj / alpha * lvs[j];
        a.host[j] = hj;
        a.host[kHostWW] = sums[nv];   // w . w
        if (j > 0) a.vs[j] = 1.0;   // S_j is rewritten as the unit vector v_j
    } else if (a.mode == 6) {
        // after the update (sums: S_i . w1 for i < j, v_j . w1, w1 . w1):
        // beta = |w1|, p_{j+1} = w1 / beta, a_i = v_i . p_{j+1} (i <= j)
        const int j = nv - 1;
        const double beta = sqrt(fmax(sums[nv], 0.0));
        const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
        a.vs[nv] = inv;
        for (int i = 0; i <= j; ++i) {
            const double ai = (i < j ? lvs[i] : 1.0) * sums[i] * inv;
            a.a[i] = ai;
            a.host[kHostA + i] = ai;
        }
        a.host[nv] = beta;
    } else if (a.mode == 0) {
        for (int i = 0; i < nv; ++i) {
            const double h = lvs[i] * sums[i];
            a.h1[i] = h;
            a.c[i] = lvs[i] * h;
        }
    } else if (a.mode == 1) {
        for (int i = 0; i < nv; ++i) {
            const double h = lvs[i] * sums[i];
            a.h2[i] = h;
            a.c[i] = lc[i] + lvs[i] * h;
        }
    } else if (a.mode == 2 || a.mode == 3) {
        const double nrm = sqrt(fmax(sums[0], 0.0));
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        if (a.mode == 2) {
            a.vs[nv] = inv;
            for (int i = 0; i < nv; ++i) a.host[i] = lh1[i] + lh2[i];
            a.host[nv] = nrm;
        } else {
            a.vs[0] = inv;
            a.host[kHostBeta] = nrm;
        }
    } else {
        a.host[kHostBB] = sums[0];
        if (nv == 1) {
            const double nrm = sqrt(fmax(sums[0], 0.0));
            a.vs[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
            a.host[kHostBeta] = nrm;
        }
    }
    a.host[kHostFail] = (a.fail && *a.fail) ? 1.0 : 0.0;
    // the host may poll the sequence number instead of synchronising the stream
    __threadfence_system();
    a.host[kHostSeq] = a.seq;
}

hipError_t launch_reduce_small(const double *part, int nblk, int ldp, const SmallArgs &a,
                               hipStream_t st)
{
    k_reduce_small<<<1, 1024, 0, st>>>(part, nblk, ldp, a);
    return hipGetLastError();
}

}  // namespace aao
