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
#include "aao_internal.h"

namespace aao {

// ------------------------------------------------------------ sine transform
// out[k][p][i] = sqrt(2/(ny+1)) sum_q in[k][q][i] sin(pi p q/(ny+1)), p, q = 1..ny.
// Two neighbouring columns (a, b) of a level form one complex sequence v = a + i b.
// Its odd extension z of length Ly = 2(ny+1) (z_0 = z_{ny+1} = 0, z_q = v_q,
// z_{Ly-q} = -v_q) has the DFT Z_p = -2i (A_p + i B_p), A and B the unnormalised sine
// transforms of a and b, so A_p = -Im Z_p / 2 and B_p = Re Z_p / 2.
// One workgroup holds S sequences (2S columns of one level) and a twiddle table in
// LDS and transforms them with radix-4 Stockham passes (a last radix-2 pass when
// log2 Ly is odd), in place: each pass reads all its inputs into registers, waits,
// then writes.
constexpr int kDstThreads = 256;
constexpr int kDstElems = 4096;                          // complex sequence entries per workgroup
constexpr int kDstVals = kDstElems / kDstThreads;        // per thread and pass

bool dst_y_supported(int ny) { return ny >= 1 && ny <= 2047 && ((ny + 1) & ny) == 0; }

static int dst_seqs(int nx, int ny)
{
    const int Ly = 2 * (ny + 1);
    int S = kDstElems / Ly;
    if (S > 32) S = 32;
    const int need = (nx + 1) / 2;
    if (S > need) S = need;
    return S < 1 ? 1 : S;
}

template <int R>
__device__ __forceinline__ void dft_small(cx<double> (&v)[R])
{
    if (R == 2) {
        const cx<double> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    } else {
        // forward radix 4: factors (-i)^{rs}
        const cx<double> t0 = v[0] + v[2], t1 = v[0] - v[2];
        const cx<double> t2 = v[1] + v[3], t3 = v[1] - v[3];
        v[0] = t0 + t2;
        v[2] = t0 - t2;
        v[1] = t1 - mul_i(t3);
        v[3] = t1 + mul_i(t3);
    }
}

// One Stockham pass of radix R over S sequences of length Ly held in buf, for
// sub-transform length Ns: butterfly j (< Ly/R) of sequence s reads entries
// j + r Ly/R, multiplies entry r by w^{r (j mod Ns) Ly/(Ns R)} (w = exp(-2 pi i/Ly)),
// transforms them and writes entry r to (j / Ns) Ns R + (j mod Ns) + r Ns.
template <int R>
__device__ __forceinline__ void dst_pass(cx<double> *buf, const cx<double> *tw, int S, int Ly,
                                         int lgLy, int Ns, int lgNs)
{
    constexpr int IT = kDstVals / R;   // butterflies per thread
    const int lgnb = lgLy - (R == 4 ? 2 : 1);
    const int nb = 1 << lgnb;
    const int items = S << lgnb;
    const int tws = Ly >> (lgNs + (R == 4 ? 2 : 1));
    cx<double> v[IT][R];
    int dst[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = threadIdx.x + it * kDstThreads;
        dst[it] = -1;
        if (b < items) {
            const int s = b >> lgnb;
            const int j = b & (nb - 1);
            const int jm = j & (Ns - 1);
            const cx<double> *src = buf + (size_t)s * Ly + j;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const cx<double> x = src[r * nb];
                v[it][r] = r == 0 ? x : x * tw[r * jm * tws];
            }
            dft_small<R>(v[it]);
            dst[it] = s * Ly + ((j >> lgNs) << lgNs) * R + jm;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        if (dst[it] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[it] + r * Ns] = v[it][r];
        }
    }
    __syncthreads();
}

// grid (ceil(nx / 2S), ell); in == out allowed (a workgroup reads its whole tile
// before it writes, and tiles are disjoint)
__global__ void __launch_bounds__(kDstThreads)
k_dst_y(const double *in, double *out, int nx, int ny, int S)
{
    extern __shared__ unsigned char dsm_raw[];
    const int Ly = 2 * (ny + 1);
    const int lgLy = 31 - __builtin_clz(Ly);
    cx<double> *buf = reinterpret_cast<cx<double> *>(dsm_raw);
    cx<double> *tw = buf + (size_t)S * Ly;
    const int t = threadIdx.x;
    const int TX = 2 * S;
    const int x0 = blockIdx.x * TX;
    const size_t lvl = (size_t)blockIdx.y * ny * nx;

    // the tile (ny rows of TX columns), all loads in flight before any LDS store
    const int tot = ny * TX;
    double val[kDstVals];
#pragma unroll
    for (int k = 0; k < kDstVals; ++k) {
        const int e = t + k * kDstThreads;
        const int q = e / TX, c = e - q * TX;
        const bool ok = e < tot && x0 + c < nx;
        val[k] = ok ? in[lvl + (size_t)q * nx + x0 + c] : 0.0;
    }
    for (int p = t; p < Ly; p += kDstThreads) {
        double sn, cs;
        sincospi(-2.0 * (double)p / (double)Ly, &sn, &cs);
        tw[p] = {cs, sn};
    }
    for (int s = t; s < S; s += kDstThreads) {
        buf[(size_t)s * Ly] = {0.0, 0.0};
        buf[(size_t)s * Ly + ny + 1] = {0.0, 0.0};
    }
    double *bd = reinterpret_cast<double *>(buf);
#pragma unroll
    for (int k = 0; k < kDstVals; ++k) {
        const int e = t + k * kDstThreads;
        if (e < tot) {
            const int q = e / TX, c = e - q * TX;
            const size_t base = 2 * (size_t)(c >> 1) * Ly + (c & 1);
            bd[base + 2 * (q + 1)] = val[k];
            bd[base + 2 * (Ly - q - 1)] = -val[k];
        }
    }
    __syncthreads();

    int Ns = 1, lgNs = 0;
    while (lgNs + 2 <= lgLy) {
        dst_pass<4>(buf, tw, S, Ly, lgLy, Ns, lgNs);
        Ns <<= 2;
        lgNs += 2;
    }
    if (lgNs < lgLy) dst_pass<2>(buf, tw, S, Ly, lgLy, Ns, lgNs);

    const double f = 0.5 * sqrt(2.0 / (ny + 1.0));
#pragma unroll
    for (int k = 0; k < kDstVals; ++k) {
        const int e = t + k * kDstThreads;
        const int q = e / TX, c = e - q * TX;
        if (e < tot && x0 + c < nx) {
            const cx<double> z = buf[(size_t)(c >> 1) * Ly + q + 1];
            out[lvl + (size_t)q * nx + x0 + c] = (c & 1) ? f * z.x : -f * z.y;
        }
    }
}

hipError_t launch_dst_y(const double *in, double *out, int nx, int ny, int ell, hipStream_t st)
{
    if (!dst_y_supported(ny) || nx < 1 || ell < 1 || ell > 65535) return hipErrorInvalidValue;
    const int S = dst_seqs(nx, ny);
    const int Ly = 2 * (ny + 1);
    const size_t smem = sizeof(cx<double>) * ((size_t)S * Ly + Ly);
    if (smem > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_dst_y,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    dim3 grid((nx + 2 * S - 1) / (2 * S), ell);
    k_dst_y<<<grid, kDstThreads, smem, st>>>(in, out, nx, ny, S);
    return hipGetLastError();
}

// ------------------------------------------------------------ Q1 stencils
// P = M2 x and Q = K2 x at node (iy, ix) of one level:
//   M2 = My (x) Mx:  hx hy / 36 * [1 4 1] (x) [1 4 1],
//   K2 = Ky (x) Mx + My (x) Kx:  hx/(6 hy) [-1 2 -1]_y [1 4 1]_x + hy/(6 hx) [1 4 1]_y [-1 2 -1]_x.
// The nine loads are issued at clamped addresses and masked.
__device__ __forceinline__ void q1_mk(const double *__restrict__ xl, int nx, int ny, int ix,
                                      int iy, double hx, double hy, double &P, double &Q)
{
    const int il = ix > 0 ? ix - 1 : 0, ir = ix < nx - 1 ? ix + 1 : ix;
    const double ml = ix > 0 ? 1.0 : 0.0, mr = ix < nx - 1 ? 1.0 : 0.0;
    double mrow[3], krow[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int yy = iy + d - 1;
        const bool ok = yy >= 0 && yy < ny;
        const double *row = xl + (size_t)(ok ? yy : iy) * nx;
        const double a = ml * row[il], b = row[ix], c = mr * row[ir];
        const double w = ok ? 1.0 : 0.0;
        mrow[d] = w * (a + 4.0 * b + c);
        krow[d] = w * (2.0 * b - a - c);
    }
    P = (hx * hy / 36.0) * (mrow[0] + 4.0 * mrow[1] + mrow[2]);
    Q = (hx / (6.0 * hy)) * (2.0 * mrow[1] - mrow[0] - mrow[2]) +
        (hy / (6.0 * hx)) * (krow[0] + 4.0 * krow[1] + krow[2]);
}

// ------------------------------------------------------------------ matvec
// y_k = sum_m (a_m M2 + b_m kappa K2) x_{k-m} (start-up rows and the block above the
// diagonal through scheme_block), or the transpose y_k = sum_m A_{k+m,k} x_{k+m}
// (every block symmetric).  A thread owns one node and walks a segment of TS time
// levels (upwards, or downwards for the transpose), keeping M2 x and K2 x of the W
// levels its rows touch in registers: window slot c holds level k - dir (c - up).
constexpr int kMv2Seg = 32;

template <int W>
__global__ void __launch_bounds__(256)
k_matvec2d(const double *__restrict__ x, double *__restrict__ y, const double *__restrict__ bsub,
           int nx, int ny, int ell, Scheme sc, double kappa, int transpose)
{
    const int ix = blockIdx.x * 64 + (threadIdx.x & 63);
    const int iy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (ix >= nx || iy >= ny) return;
    const int up = sc.up;
    const int dir = transpose ? -1 : 1;
    const int kb = blockIdx.z * kMv2Seg;
    const int ke = min(ell, kb + kMv2Seg);
    const int k0 = transpose ? ke - 1 : kb;
    const int cnt = ke - kb;
    const size_t lv = (size_t)nx * ny;
    const double hx = 1.0 / (nx + 1.0), hy = 1.0 / (ny + 1.0);
    double P[W], Q[W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const int L = k0 - dir * (c - up);
        P[c] = Q[c] = 0.0;
        if (L >= 0 && L < ell) q1_mk(x + (size_t)L * lv, nx, ny, ix, iy, hx, hy, P[c], Q[c]);
    }
    const size_t node = (size_t)iy * nx + ix;
    for (int t = 0; t < cnt; ++t) {
        const int k = k0 + dir * t;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const int m = c - up;
            const int src = transpose ? k + m : k - m;
            const int row = transpose ? src : k;
            double cm, cb;
            if (src >= 0 && src < ell && scheme_block(sc, row, m, cm, cb))
                acc += cm * P[c] + cb * kappa * Q[c];
        }
        const size_t o = (size_t)k * lv + node;
        y[o] = bsub ? bsub[o] - acc : acc;
        if (t + 1 < cnt) {
#pragma unroll
            for (int c = W - 1; c > 0; --c) {
                P[c] = P[c - 1];
                Q[c] = Q[c - 1];
            }
            const int L = k + dir + dir * up;
            P[0] = Q[0] = 0.0;
            if (L >= 0 && L < ell) q1_mk(x + (size_t)L * lv, nx, ny, ix, iy, hx, hy, P[0], Q[0]);
        }
    }
}

hipError_t launch_matvec2d(const double *x, double *y, const double *bsub, int nx, int ny,
                           int ell, Scheme sc, double kappa, int transpose, hipStream_t st)
{
    dim3 grid((nx + 63) / 64, (ny + 3) / 4, (ell + kMv2Seg - 1) / kMv2Seg);
    switch (sc.s + sc.up + 1) {
    case 2: k_matvec2d<2><<<grid, 256, 0, st>>>(x, y, bsub, nx, ny, ell, sc, kappa, transpose); break;
    case 3: k_matvec2d<3><<<grid, 256, 0, st>>>(x, y, bsub, nx, ny, ell, sc, kappa, transpose); break;
    case 4: k_matvec2d<4><<<grid, 256, 0, st>>>(x, y, bsub, nx, ny, ell, sc, kappa, transpose); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------- right-hand side
// Heat: b_0 = M2 u0.  BD2: b_0 = (M2 + tau^2 kappa K2)(u0 + tau v0), b_1 = -M2 u0
// (v0 = 0 if absent).  Every later row is zero.
__global__ void __launch_bounds__(256)
k_rhs2d(double *__restrict__ b, const double *__restrict__ u0, const double *__restrict__ v0,
        int nx, int ny, int ell, int scheme, double tau, double kappa)
{
    const int ix = blockIdx.x * 64 + (threadIdx.x & 63);
    const int iy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (ix >= nx || iy >= ny) return;
    const double hx = 1.0 / (nx + 1.0), hy = 1.0 / (ny + 1.0);
    const size_t lv = (size_t)nx * ny, node = (size_t)iy * nx + ix;
    double Pu, Qu;
    q1_mk(u0, nx, ny, ix, iy, hx, hy, Pu, Qu);
    int k = 1;
    if (scheme == AAO_HEAT_IE) {
        b[node] = Pu;
    } else {
        double Pv = 0.0, Qv = 0.0;
        if (v0) q1_mk(v0, nx, ny, ix, iy, hx, hy, Pv, Qv);
        b[node] = (Pu + tau * Pv) + tau * tau * kappa * (Qu + tau * Qv);
        b[lv + node] = -Pu;
        k = 2;
    }
    for (; k < ell; ++k) b[(size_t)k * lv + node] = 0.0;
}

hipError_t launch_build_rhs2d(double *b, const double *u0, const double *v0, int nx, int ny,
                              int ell, Scheme sc, double kappa, double tau, hipStream_t st)
{
    if (sc.id != AAO_HEAT_IE && (sc.id != AAO_WAVE_BD2 || ell < 2)) return hipErrorInvalidValue;
    dim3 grid((nx + 63) / 64, (ny + 3) / 4);
    k_rhs2d<<<grid, 256, 0, st>>>(b, u0, v0, nx, ny, ell, sc.id, tau, kappa);
    return hipGetLastError();
}

}  // namespace aao
