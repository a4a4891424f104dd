// The all-at-once method on the unit square: bilinear (Q1) elements on a uniform
// nx x ny interior grid, zero Dirichlet data.  The paper works in one space dimension
// and notes (Sec. 3 and Sec. 5) that with more dimensions the blocks of the
// preconditioner's middle factor are no longer tridiagonal.  On a tensor-product grid
// they still reduce to tridiagonal ones: M2 = My (x) Mx and K2 = Ky (x) Mx + My (x) Kx,
// and the orthonormal sine transform S_y diagonalises My and Ky, so
//   (I (x) S_y (x) I) (alpha M2 + beta kappa K2) (I (x) S_y (x) I)
//     = blockdiag_q ((alpha my_q + beta kappa ky_q) Mx + beta kappa my_q Kx),
// one x-tridiagonal per (frequency, sine mode) pair, solved by the same partition
// solve as in one dimension.  C^{-1} r = S_y F^{-1} [solves] F S_y r, where the time
// transform F and S_y act on different axes and commute.
//
// This file: the sine transform along y, the block-Toeplitz matvec with the Q1
// stencils, and the right-hand side.  All FP64 and memory-bound.
#include "../../include/aao.h"
#include "fft_core.h"

namespace aao {

// ------------------------------------------------------------ sine transform
// out[k][p][i] = sqrt(2/N) sum_q in[k][q][i] sin(pi p q / N), p, q = 1..ny, N = ny + 1.
// A length-N transform per column (half the length of the odd extension), by the
// sine-weighted fold of the sequence with its mirror:
//   y_0 = 0,  y_q = sin(pi q/N) (f_q + f_{N-q}) + (f_q - f_{N-q}) / 2,  q = 1..N-1,
// whose DFT Y_k = sum_q y_q exp(2 pi i q k/N) gives, for real f,
//   S_{2k} = Im Y_k,   S_{2k+1} - S_{2k-1} = Re Y_k  (S_{-1} = -S_1),
// since the symmetric part of y carries only cosines and the antisymmetric part only
// sines, and 2 sin(pi q/N) cos(2 pi q k/N) = sin(pi q (2k+1)/N) - sin(pi q (2k-1)/N).
// The odd coefficients are therefore a running sum over k.  Two neighbouring real
// columns (a, b) of a level go through one complex transform as f = a + i b; with
// Z the forward DFT of y (exp(-2 pi i q k/N)), Y_k = Z_{N-k}, and the two real
// spectra separate by the conjugate symmetry Y^a_k = (Y_k + conj Y_{N-k}) / 2,
// Y^b_k = (Y_k - conj Y_{N-k}) / (2 i):
//   2 S^a_{2k} = Im Z_{N-k} - Im Z_k,   2 S^b_{2k} = Re Z_k - Re Z_{N-k},
//   2 S^a_{2k+1} = sum_{j<=k} d^a_j,  d^a_j = Re Z_j + Re Z_{N-j} (j >= 1), d^a_0 = Re Z_0,
// and likewise d^b with the imaginary parts.
// The transform along y has the shape of the time-axis transforms (a strided axis,
// contiguous columns), so it runs on the same register-resident Stockham machinery
// (radix 8): a workgroup owns W complex columns (2W real columns, one row segment of
// 16 W bytes per row) of one level, thread (t, c) holds P points of column c.  The
// rows enter through LDS in whole row segments, so each is read from memory once and
// the mirrored reads of the fold come from LDS.  After the transform the spectrum
// goes to LDS once more; thread (t, c) then owns k = tK .. tK + K - 1 (K = P/2): the
// even outputs and its part of the running sum, completed by a shuffle scan over the
// threads of its column in the wave and the totals of the waves before it.
bool dst_y_supported(int ny) { return ny >= 1 && ny <= 2047 && ((ny + 1) & ny) == 0; }

template <int N>
constexpr int dst_points() { return N < 8 ? N : 8; }

// LDS bytes of a workgroup of W complex columns: the staged rows ((N - 1) 2W doubles),
// one exchange plane (lds_rows(N) W doubles) and the spectrum (rows k + k/8 < N + N/8,
// W complex each) plus the per-wave running-sum totals share one buffer.
static size_t dst_lds(int N, int W)
{
    const int P = N < 8 ? N : 8;
    const int waves = (W * (N / P) + 63) / 64;
    const size_t stage = (size_t)(N - 1) * 2 * W * 8;
    const size_t plane = (size_t)(N + N / 16 + 1) * W * 8;
    const size_t spec = ((size_t)(N + N / 8 + 1) + waves) * W * 16;
    return stage > plane ? (stage > spec ? stage : spec) : (plane > spec ? plane : spec);
}

template <int N>
__global__ void __launch_bounds__(1024)
k_dst_y(const double *in, double *out, int nx, int ell, int W, const cx<double> *__restrict__ tw)
{
    constexpr int P = dst_points<N>(), TN = N / P, K = P / 2 > 0 ? P / 2 : 1, ny = N - 1;
    extern __shared__ unsigned char dsm_raw[];
    double *sm = reinterpret_cast<double *>(dsm_raw);
    const int NT = blockDim.x;
    const int c = threadIdx.x % W;
    const int t = threadIdx.x / W;
    const int tiles_x = (nx + 2 * W - 1) / (2 * W);
    const int g = xcd_tile(blockIdx.x, gridDim.x);
    const int lvl = g / tiles_x;
    if (lvl >= ell) return;                       // padding workgroup: no barrier reached
    const int xb = (g - lvl * tiles_x) * 2 * W;   // first real column of the tile
    const int W2 = 2 * W, lw2 = __ffs(W2) - 1;    // W is a power of two
    const size_t base = (size_t)lvl * ny * nx;
    // The tile's ny rows of 2W doubles pass through LDS (row q at sm[q * 2W]):
    // ny * 2W < 2P * NT, so 2P passes cover it, in groups of eight loads (all in
    // flight, then written).
    constexpr int NL = 2 * P;
    constexpr int GL = NL < 8 ? NL : 8;
#pragma unroll
    for (int u0 = 0; u0 < NL; u0 += GL) {
        double val[GL];
#pragma unroll
        for (int u = 0; u < GL; ++u) {
            const int e = threadIdx.x + (u0 + u) * NT;
            const int q = min(e >> lw2, ny - 1), x = min(xb + (e & (W2 - 1)), nx - 1);
            val[u] = in[base + (size_t)q * nx + x];   // clamped: issued unconditionally
        }
#pragma unroll
        for (int u = 0; u < GL; ++u) {
            const int e = threadIdx.x + (u0 + u) * NT;
            if (e < ny * W2) sm[e] = xb + (e & (W2 - 1)) < nx ? val[u] : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // the fold: rows q - 1 and N - q - 1 of the column pair, sin(pi q/N) = -Im tw[q]
    // (tw holds exp(-2 pi i k / 2N))
    const double2 *rows = reinterpret_cast<const double2 *>(sm);
    cx<double> v[P];
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        const int q = first_pos<N, P>(t, idx);
        const bool data = q >= 1;
        const double2 fq = rows[(data ? q - 1 : 0) * W + c];
        const double2 fm = rows[(data ? N - q - 1 : 0) * W + c];
        const double s = data ? -tw[q].y : 0.0, h = data ? 0.5 : 0.0;
        v[idx] = {s * (fq.x + fm.x) + h * (fq.x - fm.x), s * (fq.y + fm.y) + h * (fq.y - fm.y)};
    }
    __syncthreads();                               // staging read before the first exchange
    run_stages<double, N, P, 0, false>(v, sm, t, c, W, tw, 2);
    // spectrum to LDS (every exchange read has passed its barrier)
    double2 *zs = reinterpret_cast<double2 *>(sm);
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        const int k = final_pos<N, P>(t, idx);
        zs[(k + (k >> 3)) * W + c] = make_double2(v[idx].x, v[idx].y);
    }
    __syncthreads();
    double ea[K], eb[K], pa[K], pb[K];
    double ra = 0.0, rb = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int k = t * K + i, km = (N - k) & (N - 1);
        const double2 z = zs[(k + (k >> 3)) * W + c];
        const double2 zm = zs[(km + (km >> 3)) * W + c];
        ea[i] = zm.y - z.y;
        eb[i] = z.x - zm.x;
        const double w = k == 0 ? 0.5 : 1.0;       // d_0 = Re / Im Z_0
        ra += w * (z.x + zm.x);
        rb += w * (z.y + zm.y);
        pa[i] = ra;
        pb[i] = rb;
    }
    // inclusive scan of the thread sums over t: the threads of column c sit W lanes apart
    const int lane = threadIdx.x & 63;
    double sa = ra, sb = rb;
    for (int d = W; d < 64; d <<= 1) {
        const double oa = __shfl_up(sa, d, 64), ob = __shfl_up(sb, d, 64);
        if (lane >= d) {
            sa += oa;
            sb += ob;
        }
    }
    double xa = sa - ra, xb2 = sb - rb;             // exclusive within the wave
    if (NT > 64) {                                  // uniform over the workgroup
        double2 *wt = zs + (N + N / 8 + 1) * W;
        const int wv = threadIdx.x >> 6;
        if (lane >= 64 - W) wt[wv * W + c] = make_double2(sa, sb);
        __syncthreads();
        for (int w2 = 0; w2 < wv; ++w2) {
            const double2 o = wt[w2 * W + c];
            xa += o.x;
            xb2 += o.y;
        }
    }
    const double f = 0.5 * sqrt(2.0 / N);
    const int x0 = xb + 2 * c;
    const bool ha = x0 < nx, hb = x0 + 1 < nx;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int k = t * K + i;
        if (k >= 1) {                               // p = 2k
            const size_t o = base + (size_t)(2 * k - 1) * nx + x0;
            if (ha) out[o] = f * ea[i];
            if (hb) out[o + 1] = f * eb[i];
        }
        const size_t o = base + (size_t)(2 * k) * nx + x0;   // p = 2k + 1
        if (ha) out[o] = f * (xa + pa[i]);
        if (hb) out[o + 1] = f * (xb2 + pb[i]);
    }
}

// complex columns per workgroup: a 128-byte row segment where the thread and LDS
// budgets allow (at most 1024 threads; 80 KB of LDS so that two workgroups share a
// compute unit, else 160 KB), no wider than the grid needs
static int dst_cols(int N, int nx)
{
    const int P = N < 8 ? N : 8;
    const int need = (nx + 1) / 2;
    int best = 1;
    for (int W = 1; W <= 64; W *= 2) {
        const size_t lds = dst_lds(N, W);
        if (W * (N / P) > 1024 || lds > 160 * 1024) break;
        if (W > 8 && lds > 80 * 1024) break;
        best = W;
        if (W >= need) break;
    }
    return best;
}

template <int N>
static hipError_t dst_go(const double *in, double *out, int nx, int ell, const double *tw,
                         hipStream_t st)
{
    const int W = dst_cols(N, nx);
    const int threads = W * (N / dst_points<N>());
    const size_t smem = dst_lds(N, W);
    auto kern = k_dst_y<N>;
    if (smem > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    const long long tiles = (long long)((nx + 2 * W - 1) / (2 * W)) * ell;
    if (tiles > (1LL << 30)) return hipErrorInvalidValue;
    kern<<<xcd_grid((int)tiles), threads, smem, st>>>(in, out, nx, ell, W,
                                                     reinterpret_cast<const cx<double> *>(tw));
    return hipGetLastError();
}

hipError_t launch_dst_y(const double *in, double *out, int nx, int ny, int ell, const double *tw,
                        hipStream_t st)
{
    if (!dst_y_supported(ny) || nx < 1 || ell < 1 || !tw) return hipErrorInvalidValue;
    switch (ny + 1) {
    case 2: return dst_go<2>(in, out, nx, ell, tw, st);
    case 4: return dst_go<4>(in, out, nx, ell, tw, st);
    case 8: return dst_go<8>(in, out, nx, ell, tw, st);
    case 16: return dst_go<16>(in, out, nx, ell, tw, st);
    case 32: return dst_go<32>(in, out, nx, ell, tw, st);
    case 64: return dst_go<64>(in, out, nx, ell, tw, st);
    case 128: return dst_go<128>(in, out, nx, ell, tw, st);
    case 256: return dst_go<256>(in, out, nx, ell, tw, st);
    case 512: return dst_go<512>(in, out, nx, ell, tw, st);
    case 1024: return dst_go<1024>(in, out, nx, ell, tw, st);
    case 2048: return dst_go<2048>(in, out, nx, ell, tw, st);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------ Q1 stencils
// M2 x and K2 x at one node of a level, with
//   M2 = My (x) Mx:  hx hy / 36 * [1 4 1] (x) [1 4 1],
//   K2 = Ky (x) Mx + My (x) Kx:  hx/(6 hy) [-1 2 -1]_y [1 4 1]_x + hy/(6 hx) [1 4 1]_y [-1 2 -1]_x;
// the loads are issued at clamped addresses and masked.
// In sine coordinates along y (row q of a level holding the coefficient of the q-th
// sine mode) the same operators are S_y M2 S_y = diag(my_q) (x) Mx and
// S_y K2 S_y = diag(ky_q) (x) Mx + diag(my_q) (x) Kx, with
// my_q = hy/6 e_q, ky_q = (6 - e_q)/hy, e_q = 4 + 2 cos(pi q/(ny + 1)):
// a three-point stencil within the row (HAT below).

// ------------------------------------------------------------------ matvec
// y_k = sum_m (a_m M2 + b_m kappa K2) x_{k-m} (start-up rows and the block above the
// diagonal through scheme_block), or the transpose y_k = sum_m A_{k+m,k} x_{k+m}
// (every block symmetric); y = bsub - A x if bsub.  A thread owns MR consecutive
// nodes of one x-column and walks a segment of kMv2Seg time levels (upwards, or
// downwards for the transpose), keeping M2 x and K2 x of the W levels its rows touch
// in registers: window slot c holds level k - dir (c - up).  The MR + 2 rows of a
// level are loaded together (MR independent outputs per step keep enough loads in
// flight), and the vertical stencil shares them.
//
// The GMRES forms of the launch (as in one dimension; GMRES on the unit square runs in
// sine coordinates, so these exist for the HAT stencils only): DOTS = 1 also leaves the block
// partials of V_q . y (q < nv) and of y . y (value nv), the first Gram-Schmidt pass;
// DOTS = 2 the partial of y . y only (a residual norm).  Partials are value-major,
// part[q ldp + block].  The rows of bsub and of the first kMv2DotG basis vectors that
// the next level needs are loaded with that level's x rows, so their latency overlaps
// the stencil's, and their dot products accumulate while the segment is walked; basis
// vectors past kMv2DotG are dotted after the walk with y read back, so those launches
// need y.  Without the halo rows of the 9-point stencil two rows per thread beat four
// (92 against 97 us per launch at 511 x 511 x 64).  (Forming x = Z y inside the
// residual check, as the 1D matvec does, made the nodal kernel slower than a separate
// axpy: the combination is recomputed at every neighbour of the 9-point stencil.)
constexpr int kMv2Seg = 8;
constexpr int kMv2Rows = 4;     // plain launch
constexpr int kMv2RowsDot = 2;  // launches with dot products
constexpr int kMv2DotG = 2;     // basis vectors dotted during the walk

int matvec2d_dot_walk() { return kMv2DotG; }

int matvec2d_blocks(int nx, int ny, int ell, bool dots)
{
    const int mr = dots ? kMv2RowsDot : kMv2Rows;
    return ((nx + 63) / 64) * ((ny + 4 * mr - 1) / (4 * mr)) * ((ell + kMv2Seg - 1) / kMv2Seg);
}

// the (MR + 2) x 3 neighbourhood of nodes (iy0 + o, ix), o < MR, of the level of x
// at offset lofs; loads at clamped addresses, masked
template <int MR, bool HAT = false>
__device__ __forceinline__ void q1_load(const double *__restrict__ x, size_t lofs, int nx, int ny,
                                        int ix, int iy0, double (&v)[MR + 2][3])
{
    const int il = ix > 0 ? ix - 1 : 0, ir = ix < nx - 1 ? ix + 1 : ix;
    const double ml = ix > 0 ? 1.0 : 0.0, mr = ix < nx - 1 ? 1.0 : 0.0;
#pragma unroll
    for (int d = 0; d < MR + 2; ++d) {
        if (HAT && (d == 0 || d == MR + 1)) {     // no coupling between sine modes
            v[d][0] = v[d][1] = v[d][2] = 0.0;
            continue;
        }
        const int yy = iy0 + d - 1;
        const double w = (yy >= 0 && yy < ny) ? 1.0 : 0.0;
        const size_t ro = lofs + (size_t)((yy >= 0 && yy < ny) ? yy : 0) * nx;
        v[d][0] = w * ml * x[ro + il];
        v[d][1] = w * x[ro + ix];
        v[d][2] = w * mr * x[ro + ir];
    }
}

// M2 x and K2 x at the MR nodes from their neighbourhood (Q1 stencils above)
template <int MR>
__device__ __forceinline__ void q1_apply(const double (&v)[MR + 2][3], double hx, double hy,
                                         double (&P)[MR], double (&Q)[MR])
{
    double mrow[MR + 2], krow[MR + 2];
#pragma unroll
    for (int d = 0; d < MR + 2; ++d) {
        mrow[d] = v[d][0] + 4.0 * v[d][1] + v[d][2];
        krow[d] = 2.0 * v[d][1] - v[d][0] - v[d][2];
    }
    const double cm = hx * hy / 36.0, ck1 = hx / (6.0 * hy), ck2 = hy / (6.0 * hx);
#pragma unroll
    for (int o = 0; o < MR; ++o) {
        P[o] = cm * (mrow[o] + 4.0 * mrow[o + 1] + mrow[o + 2]);
        Q[o] = ck1 * (2.0 * mrow[o + 1] - mrow[o] - mrow[o + 2]) +
               ck2 * (krow[o] + 4.0 * krow[o + 1] + krow[o + 2]);
    }
}

// the same in sine coordinates along y: e[o] = 4 + 2 cos(pi (iy0 + o + 1)/(ny + 1))
template <int MR>
__device__ __forceinline__ void q1_apply_hat(const double (&v)[MR + 2][3], double hx, double hy,
                                             const double (&e)[MR], double (&P)[MR],
                                             double (&Q)[MR])
{
    const double cm = hx * hy / 36.0, ck1 = hx / (6.0 * hy), ck2 = hy / (6.0 * hx);
#pragma unroll
    for (int o = 0; o < MR; ++o) {
        const double mrow = v[o + 1][0] + 4.0 * v[o + 1][1] + v[o + 1][2];
        const double krow = 2.0 * v[o + 1][1] - v[o + 1][0] - v[o + 1][2];
        P[o] = cm * e[o] * mrow;
        Q[o] = ck1 * (6.0 - e[o]) * mrow + ck2 * e[o] * krow;
    }
}

// the sine-mode factors e[o] of rows iy0 .. iy0 + MR - 1
template <int MR>
__device__ __forceinline__ void hat_modes(int iy0, int ny, double (&e)[MR])
{
#pragma unroll
    for (int o = 0; o < MR; ++o) e[o] = 4.0 + 2.0 * cospi((iy0 + o + 1.0) / (ny + 1.0));
}

// M2 x and K2 x at nodes (iy0 + o, ix), o < MR, of one level of x
template <int MR>
__device__ __forceinline__ void q1_mk_rows(const double *__restrict__ xl, int nx, int ny, int ix,
                                           int iy0, double hx, double hy, double (&P)[MR],
                                           double (&Q)[MR])
{
    double v[MR + 2][3];
    q1_load<MR>(xl, 0, nx, ny, ix, iy0, v);
    q1_apply<MR>(v, hx, hy, P, Q);
}

// sum over the workgroup of one value per thread, fixed order (4 waves); every thread
// gets the sum
__device__ __forceinline__ double block_sum4(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double s = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return s;
}

// The plain launch (no dot products): the window walk alone.  (Sharing the dot forms
// body, with its per-level fetches, made this launch a third slower.)
template <int W, int MR, bool HAT>
__global__ void __launch_bounds__(256)
k_matvec2d_plain(const double *__restrict__ x, double *__restrict__ y,
                 const double *__restrict__ bsub, int nx, int ny, int ell, Scheme sc,
                 double kappa, int transpose)
{
    const int ix = blockIdx.x * 64 + (threadIdx.x & 63);
    const int iy0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * MR;
    if (ix >= nx || iy0 >= ny) return;
    const int up = sc.up;
    const int dir = transpose ? -1 : 1;
    const int kb = blockIdx.z * kMv2Seg;
    const int ke = min(ell, kb + kMv2Seg);
    const int k0 = transpose ? ke - 1 : kb;
    const int cnt = ke - kb;
    const size_t lv = (size_t)nx * ny;
    const double hx = 1.0 / (nx + 1.0), hy = 1.0 / (ny + 1.0);
    double e[MR];
    if (HAT) hat_modes<MR>(iy0, ny, e);
    double P[W][MR], Q[W][MR];
    auto fill = [&](int c, int L) {
#pragma unroll
        for (int o = 0; o < MR; ++o) P[c][o] = Q[c][o] = 0.0;
        if (L >= 0 && L < ell) {
            double v[MR + 2][3];
            q1_load<MR, HAT>(x, (size_t)L * lv, nx, ny, ix, iy0, v);
            if (HAT) q1_apply_hat<MR>(v, hx, hy, e, P[c], Q[c]);
            else q1_apply<MR>(v, hx, hy, P[c], Q[c]);
        }
    };
#pragma unroll
    for (int c = 0; c < W; ++c) fill(c, k0 - dir * (c - up));
    for (int t = 0; t < kMv2Seg; ++t) {
        if (t >= cnt) break;
        const int k = k0 + dir * t;
        double acc[MR];
#pragma unroll
        for (int o = 0; o < MR; ++o) acc[o] = 0.0;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const int m = c - up;
            const int src = transpose ? k + m : k - m;
            const int row = transpose ? src : k;
            double cm, cb2;
            if (src >= 0 && src < ell && scheme_block(sc, row, m, cm, cb2)) {
                const double ck = cb2 * kappa;
#pragma unroll
                for (int o = 0; o < MR; ++o) acc[o] += cm * P[c][o] + ck * Q[c][o];
            }
        }
#pragma unroll
        for (int o = 0; o < MR; ++o) {
            const bool own = iy0 + o < ny;
            const size_t off = (size_t)k * lv + (size_t)(own ? iy0 + o : 0) * nx + ix;
            const double out = bsub ? (own ? bsub[off] : 0.0) - acc[o] : acc[o];
            if (own) y[off] = out;
        }
        if (t + 1 < cnt) {
#pragma unroll
            for (int c = W - 1; c > 0; --c)
#pragma unroll
                for (int o = 0; o < MR; ++o) {
                    P[c][o] = P[c - 1][o];
                    Q[c][o] = Q[c - 1][o];
                }
            fill(0, k + dir + dir * up);
        }
    }
}

// The GMRES forms (DOTS = 1 or 2).
template <int W, int MR, int DOTS, bool HAT>
__global__ void __launch_bounds__(256)
k_matvec2d(const double *__restrict__ x, double *__restrict__ y, const double *__restrict__ bsub,
           int nx, int ny, int ell, Scheme sc, double kappa, int transpose, VecList V, int nv,
           double *__restrict__ part, int ldp)
{
    constexpr int G = DOTS == 1 ? kMv2DotG : 1;
    const int ix = blockIdx.x * 64 + (threadIdx.x & 63);
    const int iy0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * MR;
    const bool live = ix < nx && iy0 < ny;   // every thread stays for the sums
    const int up = sc.up;
    const int dir = transpose ? -1 : 1;
    const int kb = blockIdx.z * kMv2Seg;
    const int ke = min(ell, kb + kMv2Seg);
    const int k0 = transpose ? ke - 1 : kb;
    const int cnt = ke - kb;
    const size_t lv = (size_t)nx * ny;
    const double hx = 1.0 / (nx + 1.0), hy = 1.0 / (ny + 1.0);
    const int ng = DOTS == 1 ? min(nv, G) : 0;
    bool own[MR];
    size_t nofs[MR];                      // node offsets within a level
#pragma unroll
    for (int o = 0; o < MR; ++o) {
        own[o] = live && iy0 + o < ny;
        nofs[o] = (size_t)(own[o] ? iy0 + o : 0) * nx + (own[o] ? ix : 0);
    }
    double e[MR];
    if (HAT) hat_modes<MR>(iy0, ny, e);
    double P[W][MR], Q[W][MR];
    auto fill = [&](int c, int L) {
#pragma unroll
        for (int o = 0; o < MR; ++o) P[c][o] = Q[c][o] = 0.0;
        if (live && L >= 0 && L < ell) {
            double v[MR + 2][3];
            q1_load<MR, HAT>(x, (size_t)L * lv, nx, ny, ix, iy0, v);
            if (HAT) q1_apply_hat<MR>(v, hx, hy, e, P[c], Q[c]);
            else q1_apply<MR>(v, hx, hy, P[c], Q[c]);
        }
    };
    // rows of bsub and of the first G basis vectors at level k (zero where not owned)
    double bc[MR], vc[G][MR];
    auto fetch = [&](int k) {
#pragma unroll
        for (int o = 0; o < MR; ++o) {
            const size_t off = (size_t)k * lv + nofs[o];
            bc[o] = (bsub && own[o]) ? bsub[off] : 0.0;
#pragma unroll
            for (int g = 0; g < G; ++g) vc[g][o] = (g < ng && own[o]) ? V.p[g][off] : 0.0;
        }
    };
#pragma unroll
    for (int c = 0; c < W; ++c) fill(c, k0 - dir * (c - up));
    if (cnt > 0) fetch(k0);
    double yy = 0.0, ad[G];
#pragma unroll
    for (int g = 0; g < G; ++g) ad[g] = 0.0;
    for (int t = 0; t < kMv2Seg; ++t) {
        if (t >= cnt) break;
        const int k = k0 + dir * t;
        double acc[MR];
#pragma unroll
        for (int o = 0; o < MR; ++o) acc[o] = 0.0;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const int m = c - up;
            const int src = transpose ? k + m : k - m;
            const int row = transpose ? src : k;
            double cm, cb2;
            if (src >= 0 && src < ell && scheme_block(sc, row, m, cm, cb2)) {
                const double ck = cb2 * kappa;
#pragma unroll
                for (int o = 0; o < MR; ++o) acc[o] += cm * P[c][o] + ck * Q[c][o];
            }
        }
#pragma unroll
        for (int o = 0; o < MR; ++o) {
            const size_t off = (size_t)k * lv + nofs[o];
            const double out = own[o] ? (bsub ? bc[o] - acc[o] : acc[o]) : 0.0;
            yy += out * out;
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (DOTS == 1) ad[g] += vc[g][o] * out;
            if (own[o] && y) y[off] = out;
        }
        if (t + 1 < cnt) {
#pragma unroll
            for (int c = W - 1; c > 0; --c)
#pragma unroll
                for (int o = 0; o < MR; ++o) {
                    P[c][o] = P[c - 1][o];
                    Q[c][o] = Q[c - 1][o];
                }
            fill(0, k + dir + dir * up);
            fetch(k + dir);
        }
    }
    __shared__ double red[4];
    const int blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    if (DOTS == 2) {
        const double s = block_sum4(yy, red);
        if (threadIdx.x == 0) part[blk] = s;
        return;
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
        if (g < ng) {
            const double s = block_sum4(ad[g], red);
            if (threadIdx.x == 0) part[(size_t)g * ldp + blk] = s;
        }
    // basis vectors past the first G: y read back (this thread wrote these entries;
    // the launcher requires y for nv > G)
    for (int q = G; q < nv; ++q) {
        double a = 0.0;
        for (int t = 0; t < cnt; ++t) {
            const size_t lo = (size_t)(k0 + dir * t) * lv;
#pragma unroll
            for (int o = 0; o < MR; ++o)
                if (own[o]) a += V.p[q][lo + nofs[o]] * y[lo + nofs[o]];
        }
        const double s = block_sum4(a, red);
        if (threadIdx.x == 0) part[(size_t)q * ldp + blk] = s;
    }
    const double s = block_sum4(yy, red);
    if (threadIdx.x == 0) part[(size_t)nv * ldp + blk] = s;
}

template <int DOTS, bool HAT>
static hipError_t matvec2d_go(const double *x, double *y, const double *bsub, int nx, int ny,
                              int ell, Scheme sc, double kappa, int transpose, const VecList &V,
                              int nv, double *part, int ldp, hipStream_t st)
{
    constexpr int MR = DOTS > 0 ? kMv2RowsDot : kMv2Rows;
    dim3 grid((nx + 63) / 64, (ny + 4 * MR - 1) / (4 * MR), (ell + kMv2Seg - 1) / kMv2Seg);
    if constexpr (DOTS == 0) {
        switch (sc.s + sc.up + 1) {
        case 2: k_matvec2d_plain<2, MR, HAT><<<grid, 256, 0, st>>>(x, y, bsub, nx, ny, ell, sc, kappa, transpose); break;
        case 3: k_matvec2d_plain<3, MR, HAT><<<grid, 256, 0, st>>>(x, y, bsub, nx, ny, ell, sc, kappa, transpose); break;
        case 4: k_matvec2d_plain<4, MR, HAT><<<grid, 256, 0, st>>>(x, y, bsub, nx, ny, ell, sc, kappa, transpose); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (sc.s + sc.up + 1) {
        case 2: k_matvec2d<2, MR, DOTS, HAT><<<grid, 256, 0, st>>>(x, y, bsub, nx, ny, ell, sc, kappa, transpose, V, nv, part, ldp); break;
        case 3: k_matvec2d<3, MR, DOTS, HAT><<<grid, 256, 0, st>>>(x, y, bsub, nx, ny, ell, sc, kappa, transpose, V, nv, part, ldp); break;
        case 4: k_matvec2d<4, MR, DOTS, HAT><<<grid, 256, 0, st>>>(x, y, bsub, nx, ny, ell, sc, kappa, transpose, V, nv, part, ldp); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}


hipError_t launch_matvec2d(const double *x, double *y, const double *bsub, int nx, int ny,
                           int ell, Scheme sc, double kappa, int transpose, hipStream_t st,
                           const VecList *V, int nv, double *part, int ldp, bool hat)
{
    static const VecList none{};
    if (nv > 0) {
        if (!V || !part || nv >= kMaxVecs || matvec2d_blocks(nx, ny, ell, true) > ldp)
            return hipErrorInvalidValue;
        if (nv > kMv2DotG && !y) return hipErrorInvalidValue;   // dots past the walk read y
        if (!hat) return hipErrorInvalidValue;   // GMRES runs in sine coordinates only
        // a one-entry list equal to the output selects the self-norm only
        if (nv == 1 && V->p[0] == y)
            return matvec2d_go<2, true>(x, y, bsub, nx, ny, ell, sc, kappa, transpose, none, 0,
                                        part, ldp, st);
        return matvec2d_go<1, true>(x, y, bsub, nx, ny, ell, sc, kappa, transpose, *V, nv, part,
                                    ldp, st);
    }
    if (!y) return hipErrorInvalidValue;
    return hat ? matvec2d_go<0, true>(x, y, bsub, nx, ny, ell, sc, kappa, transpose, none, 0,
                                      nullptr, 0, st)
               : matvec2d_go<0, false>(x, y, bsub, nx, ny, ell, sc, kappa, transpose, none, 0,
                                       nullptr, 0, st);
}

// ---------------------------------------------------------- right-hand side
// The first rows of the monolithic right-hand side, every later row zero:
//   heat b_0 = M2 u0;  BD2 b_0 = (M2 + tau^2 kappa K2)(u0 + tau v0), b_1 = -M2 u0;
//   BD4 as BD2 plus b_2 = M2 u0;  CD b_0 = -M2 u0  (v0 = 0 if absent).
__global__ void __launch_bounds__(256)
k_rhs2d(double *__restrict__ b, const double *__restrict__ u0, const double *__restrict__ v0,
        int nx, int ny, int ell, int scheme, double tau, double kappa)
{
    const int ix = blockIdx.x * 64 + (threadIdx.x & 63);
    const int iy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (ix >= nx || iy >= ny) return;
    const double hx = 1.0 / (nx + 1.0), hy = 1.0 / (ny + 1.0);
    const size_t lv = (size_t)nx * ny, node = (size_t)iy * nx + ix;
    double Pu[1], Qu[1];
    q1_mk_rows<1>(u0, nx, ny, ix, iy, hx, hy, Pu, Qu);
    int k = 1;
    if (scheme == AAO_HEAT_IE) {
        b[node] = Pu[0];
    } else if (scheme == AAO_WAVE_CD) {
        b[node] = -Pu[0];
    } else {
        double Pv[1] = {0.0}, Qv[1] = {0.0};
        if (v0) q1_mk_rows<1>(v0, nx, ny, ix, iy, hx, hy, Pv, Qv);
        b[node] = (Pu[0] + tau * Pv[0]) + tau * tau * kappa * (Qu[0] + tau * Qv[0]);
        b[lv + node] = -Pu[0];
        k = 2;
        if (scheme == AAO_WAVE_BD4) b[2 * lv + node] = Pu[0], k = 3;
    }
    for (; k < ell; ++k) b[(size_t)k * lv + node] = 0.0;
}

hipError_t launch_build_rhs2d(double *b, const double *u0, const double *v0, int nx, int ny,
                              int ell, Scheme sc, double kappa, double tau, hipStream_t st)
{
    const int rows = sc.id == AAO_WAVE_BD4 ? 3 : sc.id == AAO_WAVE_BD2 ? 2 : 1;
    if (sc.id < AAO_HEAT_IE || sc.id > AAO_WAVE_CD || ell < rows) return hipErrorInvalidValue;
    if (sc.id == AAO_WAVE_CD && v0) return hipErrorInvalidValue;
    dim3 grid((nx + 63) / 64, (ny + 3) / 4);
    k_rhs2d<<<grid, 256, 0, st>>>(b, u0, v0, nx, ny, ell, sc.id, tau, kappa);
    return hipGetLastError();
}

}  // namespace aao
