// Time-axis transforms of the circulant preconditioner apply
// (arXiv 1810.00615, Sec. 3, eq. precon2para: the (U* (x) I_n) and (U (x) I_n)
// factors, computed per spatial column as in eq. alternativecal with an FFT).
//
// Layout: the real input is ell x n row-major (row k = time level, the n
// spatial nodes contiguous), so one workgroup owns a tile of W adjacent columns
// and every global access is a W-wide row segment (coalesced across n).  No
// transpose is needed -- the paper's vector transpose is replaced by the choice
// of tile.
//
// Real-to-half-spectrum for even ell = 2L: the column is packed as the complex
// sequence z_k = x_{2k} + i x_{2k+1} of length L, transformed with a radix-16
// Stockham FFT whose data stay in registers (P points per thread) and are
// exchanged through LDS between stages (real and imaginary halves in turn, so a
// tile needs only L*W reals of LDS), then split into the half spectrum
//   X_j = (Z_j + conj Z_{L-j})/2 - (i/2) w^j (Z_j - conj Z_{L-j}),  j = 0..L,
// with w = exp(-2 pi i / ell).  The inverse runs the same steps backwards.
// Lengths that are not powers of two use a direct-DFT kernel.
#include "fft_core.h"

namespace aao {

// Forward: real ell x n (ell = 2L) -> half spectrum rows 0..L.
// Input column value at time k is r[k][col] - sigma_k kappa (K zprev_k)[col]
// when zprev != nullptr (the Neumann residual r - E z, eq. preconapprox1).
template <typename T, int L, int P, bool NEU>
__global__ void __launch_bounds__(1024)
k_fft_fwd(const double *__restrict__ r, const double *__restrict__ in_scale,
          const double *__restrict__ zprev, const double *__restrict__ sigk, double kap_h, int n,
          int W,
          cx<T> *__restrict__ X, int lds, const cx<double> *__restrict__ tw,
          double *__restrict__ norm_part)
{
    extern __shared__ unsigned char smraw[];
    __shared__ double nsum[16];
    T *sm = reinterpret_cast<T *>(smraw);
    const int c = threadIdx.x % W;
    const int t = threadIdx.x / W;
    const int col = xcd_tile(blockIdx.x, gridDim.x) * W + c;
    const bool valid = col < n;
    const double rs = in_scale ? *in_scale : 1.0;
    double nrm = 0.0;   // sum of the squared inputs (norm_part)
    cx<T> v[P];
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        const int pos = first_pos<L, P>(t, idx);
        double a = 0.0, b = 0.0;
        if (valid) {
            const size_t o0 = (size_t)(2 * pos) * n + col;
            const size_t o1 = o0 + n;
            a = r[o0];
            b = r[o1];
            nrm += a * a + b * b;
            a *= rs;
            b *= rs;
            if (NEU) {
                const double zl0 = col > 0 ? zprev[o0 - 1] : 0.0;
                const double zr0 = col < n - 1 ? zprev[o0 + 1] : 0.0;
                const double zl1 = col > 0 ? zprev[o1 - 1] : 0.0;
                const double zr1 = col < n - 1 ? zprev[o1 + 1] : 0.0;
                a -= sigk[2 * pos] * kap_h * (2.0 * zprev[o0] - zl0 - zr0);
                b -= sigk[2 * pos + 1] * kap_h * (2.0 * zprev[o1] - zl1 - zr1);
            }
        }
        v[idx] = {T(a), T(b)};
    }
    run_stages<T, L, P, 0, false>(v, sm, t, c, W, tw, 2);
    if (norm_part) {
        // block partial of ||r||^2 (unscaled input), fixed order; blocks of fewer
        // than 64 threads (short transforms) fill only part of their wave
        const int lane = threadIdx.x & 63;
        const int wl = blockDim.x < 64 ? (int)blockDim.x : 64;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_down(nrm, off, 64);
            if (lane + off < wl) nrm += o;
        }
        if (lane == 0) nsum[threadIdx.x >> 6] = nrm;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w2 = 0; w2 < (int)((blockDim.x + 63) >> 6); ++w2) s += nsum[w2];
            norm_part[blockIdx.x] = s;
        }
    }
    // Split Z into the half spectrum.  With F_e = (Z_p + conj Z_{L-p})/2,
    // F_o = (Z_p - conj Z_{L-p})/2i and w = w_ell^p:
    //   X_p = F_e + w F_o,  X_{L-p} = conj(F_e - w F_o),  X_0 = Re Z_0 + Im Z_0,
    //   X_L = Re Z_0 - Im Z_0,  X_{L/2} = conj Z_{L/2}.
    // The upper half of Z (positions L/2..L-1) goes to LDS as complex values; the
    // holders of the lower half then read their partner and write both outputs.
    constexpr int RL = Plan<L, P>::NS == 0 ? 1 : Plan<L, P>::radix(Plan<L, P>::NS - 1);
    constexpr int H2 = L / 2;
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        const int pos = final_pos<L, P>(t, idx);
        if (pos >= H2 && L > 1) {
            const int k = 2 * lds_idx(pos - H2, c, W);
            sm[k] = v[idx].x;
            sm[k + 1] = v[idx].y;
        }
    }
    __syncthreads();
    if (!valid) return;
#pragma unroll
    for (int u = 0; u < P / RL; ++u) {
        const int q = t + u * (L / P);
        const cx<double> wqd = tw[q];
        const cx<T> wq = {T(wqd.x), T(wqd.y)};
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const int idx = u * RL + r;
            const int pos = final_pos<L, P>(t, idx);
            const cx<T> z = v[idx];
            if (pos == 0) {
                X[col] = {z.x + z.y, T(0)};
                X[(size_t)L * lds + col] = {z.x - z.y, T(0)};
            } else if (2 * pos == L) {
                X[(size_t)pos * lds + col] = conj(z);
            } else if (pos < H2) {
                const int k = 2 * lds_idx(L - pos - H2, c, W);
                const cx<T> zp = {sm[k], sm[k + 1]};
                const cx<T> fe = {T(0.5) * (z.x + zp.x), T(0.5) * (z.y - zp.y)};
                const cx<T> fo = {T(0.5) * (z.y + zp.y), T(0.5) * (zp.x - z.x)};
                const cx<T> w = (r == 0) ? wq : wq * root32<false, T>(r * (16 / RL));
                const cx<T> wf = w * fo;
                X[(size_t)pos * lds + col] = fe + wf;
                X[(size_t)(L - pos) * lds + col] = conj(fe - wf);
            }
        }
    }
}

// Inverse: half spectrum rows 0..L -> real ell x n, including the 1/ell factor.
template <typename T, int L, int P>
__global__ void __launch_bounds__(1024)
k_fft_inv(const cx<T> *__restrict__ Y, int lds, double *__restrict__ z, int n, int W,
          const cx<double> *__restrict__ tw, const double *__restrict__ out_scale)
{
    extern __shared__ unsigned char smraw[];
    T *sm = reinterpret_cast<T *>(smraw);
    const int c = threadIdx.x % W;
    const int t = threadIdx.x / W;
    const int col = xcd_tile(blockIdx.x, gridDim.x) * W + c;
    const bool valid = col < n;
    cx<T> v[P];
    // E_p + i O_p with E_p = Y_p + conj Y_{L-p}, O_p = (Y_p - conj Y_{L-p}) w_ell^{-p};
    // first-stage positions are p = q + r L/R0, so w_ell^{-p} = conj(w_ell^q) times the
    // constant conj(w_{2 R0}^r)
    constexpr int R0 = Plan<L, P>::NS == 0 ? 1 : Plan<L, P>::radix(0);
#pragma unroll
    for (int u = 0; u < P / R0; ++u) {
        const int q0 = t + u * (L / P);
        const cx<double> wqd = tw[q0];
        const cx<T> wq = {T(wqd.x), T(-wqd.y)};
        // points in the order r = 0, R0-1, 1, R0-2, ...: the partner L - p of the
        // point taken in a slot is taken by its own holder in an adjacent slot, so the
        // second read of each spectrum entry comes soon after the first (from L2)
#pragma unroll
        for (int sl = 0; sl < R0; ++sl) {
            const int r = (sl & 1) ? R0 - 1 - (sl >> 1) : (sl >> 1);
            const int idx = u * R0 + r;
            const int pos = first_pos<L, P>(t, idx);
            cx<T> q = {T(0), T(0)};
            if (valid) {
                const cx<T> a = Y[(size_t)pos * lds + col];
                const cx<T> b = conj(Y[(size_t)(L - pos) * lds + col]);
                const cx<T> wc = (r == 0) ? wq : wq * root32<true, T>(r * (16 / R0));
                const cx<T> e = a + b;
                const cx<T> o = wc * (a - b);
                q = e + mul_i(o);
            }
            v[idx] = q;
        }
    }
    run_stages<T, L, P, 0, true>(v, sm, t, c, W, tw, 2);
    if (!valid) return;
    const double inv = (1.0 / (2.0 * L)) * (out_scale ? *out_scale : 1.0);
#pragma unroll
    for (int idx = 0; idx < P; ++idx) {
        const int pos = final_pos<L, P>(t, idx);
        const size_t o0 = (size_t)(2 * pos) * n + col;
        z[o0] = double(v[idx].x) * inv;
        z[o0 + n] = double(v[idx].y) * inv;
    }
}

// ---------------------------------------------------------- direct DFT path
// Any ell: X_j = sum_k x_k w^{jk}, j = 0..ell/2, one thread per (j, column).
template <typename T>
__global__ void k_dft_fwd(const double *__restrict__ r, const double *__restrict__ in_scale,
                          const double *__restrict__ zprev, const double *__restrict__ sigk,
                          double kap_h, int n, int ell,
                          cx<T> *__restrict__ X, int lds, const cx<double> *__restrict__ tw)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (col >= n) return;
    const double rs = in_scale ? *in_scale : 1.0;
    double sr = 0.0, si = 0.0;
    int p = 0;
    for (int k = 0; k < ell; ++k) {
        const size_t o = (size_t)k * n + col;
        double x = rs * r[o];
        if (zprev) {
            const double zl = col > 0 ? zprev[o - 1] : 0.0;
            const double zr = col < n - 1 ? zprev[o + 1] : 0.0;
            x -= sigk[k] * kap_h * (2.0 * zprev[o] - zl - zr);
        }
        const cx<double> w = tw[p];
        sr += x * w.x;
        si += x * w.y;
        p += j;
        if (p >= ell) p -= ell;
    }
    X[(size_t)j * lds + col] = {T(sr), T(si)};
}

// x_k = (1/ell) sum_{j=0}^{ell-1} Y_j w^{-jk} with Y_{ell-j} = conj(Y_j).
template <typename T>
__global__ void k_dft_inv(const cx<T> *__restrict__ Y, int lds, double *__restrict__ z, int n,
                          int ell, const cx<double> *__restrict__ tw)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (col >= n) return;
    const int H = ell / 2;
    double s = double(Y[col].x);
    int p = 0;
    for (int j = 1; j <= H; ++j) {
        p += k;
        if (p >= ell) p -= ell;
        const cx<T> y = Y[(size_t)j * lds + col];
        const cx<double> w = tw[p];
        // Re(y * conj(w))
        const double re = double(y.x) * w.x + double(y.y) * w.y;
        s += (2 * j == ell) ? re : 2.0 * re;
    }
    z[(size_t)k * n + col] = s / ell;
}

__global__ void k_twiddles(cx<double> *tw, int len, int count)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    const long long q = p % len;
    double s, c;
    sincospi(-2.0 * (double)q / (double)len, &s, &c);
    tw[p] = {c, s};
}

hipError_t launch_twiddles(double *tw, int len, int count, hipStream_t st)
{
    k_twiddles<<<(count + 255) / 256, 256, 0, st>>>(reinterpret_cast<cx<double> *>(tw), len,
                                                     count);
    return hipGetLastError();
}

bool fft_supported_fast(int ell) { return ell >= 2 && ell <= 16384 && (ell & (ell - 1)) == 0; }

// Launch shape of the power-of-two transforms: cfg = 16 v + log2 W, where W is the
// tile width (columns per workgroup) and v selects the points per thread P
// (v = 0: P = min(L, 16), radix-16 stages; v = 1: P = 8, radix-8 stages, offered
// for L = 512..4096).  A negative cfg selects the default.
static bool w_ok(int L, int P, int w, size_t realsz)
{
    return w >= 1 && w <= 64 && w * (L / P) <= 1024 && (size_t)w * lds_rows(L) * realsz <= 160 * 1024;
}

static int default_w(int L, int P, int n, size_t realsz)
{
    int w = 1;
    while (w < 64 && w_ok(L, P, 2 * w, realsz) && (w < 8 || w < n)) w *= 2;
    return w;
}

static bool has_p8(int L) { return L >= 512 && L <= 4096; }

int fft_configs(int ell, int n, bool single, int *out, int cap)
{
    if (!fft_supported_fast(ell)) return 0;
    const int L = ell / 2;
    const size_t rs = single ? sizeof(float) : sizeof(double);
    int k = 0;
    for (int v = 0; v < 2; ++v) {
        if (v == 1 && !has_p8(L)) break;
        const int P = v ? 8 : (L < 16 ? L : 16);
        for (int lw = 0; lw <= 6; ++lw) {
            const int w = 1 << lw;
            if (!w_ok(L, P, w, rs) || (w > 1 && (w / 2) >= n)) continue;
            if (out && k < cap) out[k] = 16 * v + lw;
            ++k;
        }
    }
    return k;
}

bool fft_config_ok(int cfg, int ell, int n, bool single)
{
    int list[16];
    const int k = fft_configs(ell, n, single, list, 16);
    for (int i = 0; i < k && i < 16; ++i)
        if (list[i] == cfg) return true;
    return false;
}

template <typename T, int L, int P>
static hipError_t fwd_LP(const double *r, const double *in_scale, const double *zprev,
                         const double *sigk, double kap_h, int n, void *spec, int lds,
                         const double *tw, hipStream_t st, int W, double *norm_part)
{
    const size_t smem = (size_t)lds_rows(L) * W * sizeof(T);
    auto kern = zprev ? k_fft_fwd<T, L, P, true> : k_fft_fwd<T, L, P, false>;
    if (smem > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    dim3 grid(xcd_grid((n + W - 1) / W));
    kern<<<grid, W * (L / P), smem, st>>>(r, in_scale, zprev, sigk, kap_h, n, W,
                                          reinterpret_cast<cx<T> *>(spec), lds,
                                          reinterpret_cast<const cx<double> *>(tw), norm_part);
    return hipGetLastError();
}

template <typename T, int L>
static hipError_t fwd_L(const double *r, const double *in_scale, const double *zprev,
                        const double *sigk, double kap_h, int n, void *spec, int lds,
                        const double *tw, hipStream_t st, int cfg, double *norm_part)
{
    constexpr int P16 = L < 16 ? L : 16;
    if (cfg >= 16) {
        if constexpr (L >= 512 && L <= 4096)
            return fwd_LP<T, L, 8>(r, in_scale, zprev, sigk, kap_h, n, spec, lds, tw, st,
                                   1 << (cfg & 15), norm_part);
        return hipErrorInvalidValue;
    }
    const int W = cfg >= 0 ? 1 << cfg : default_w(L, P16, n, sizeof(T));
    return fwd_LP<T, L, P16>(r, in_scale, zprev, sigk, kap_h, n, spec, lds, tw, st, W,
                             norm_part);
}

template <typename T, int L, int P>
static hipError_t inv_LP(const void *spec, int lds, double *z, int n, const double *tw,
                         hipStream_t st, int W, const double *out_scale)
{
    const size_t smem = (size_t)lds_rows(L) * W * sizeof(T);
    auto kern = k_fft_inv<T, L, P>;
    if (smem > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    dim3 grid(xcd_grid((n + W - 1) / W));
    kern<<<grid, W * (L / P), smem, st>>>(reinterpret_cast<const cx<T> *>(spec), lds, z, n, W,
                                          reinterpret_cast<const cx<double> *>(tw), out_scale);
    return hipGetLastError();
}

template <typename T, int L>
static hipError_t inv_L(const void *spec, int lds, double *z, int n, const double *tw,
                        hipStream_t st, int cfg, const double *out_scale)
{
    constexpr int P16 = L < 16 ? L : 16;
    if (cfg >= 16) {
        if constexpr (L >= 512 && L <= 4096)
            return inv_LP<T, L, 8>(spec, lds, z, n, tw, st, 1 << (cfg & 15), out_scale);
        return hipErrorInvalidValue;
    }
    const int W = cfg >= 0 ? 1 << cfg : default_w(L, P16, n, sizeof(T));
    return inv_LP<T, L, P16>(spec, lds, z, n, tw, st, W, out_scale);
}

template <typename T>
static hipError_t fwd_dispatch(const double *r, const double *in_scale, const double *zprev,
                               const double *sigk, double kap_h, int n, int ell, void *spec,
                               int lds, const double *tw, hipStream_t st, int cfg,
                               double *norm_part)
{
    switch (ell) {
#define AAO_CASE(E) \
    case E:                                                                                  \
        return fwd_L<T, E / 2>(r, in_scale, zprev, sigk, kap_h, n, spec, lds, tw, st, cfg,  \
                               norm_part);
        AAO_CASE(2) AAO_CASE(4) AAO_CASE(8) AAO_CASE(16) AAO_CASE(32) AAO_CASE(64)
        AAO_CASE(128) AAO_CASE(256) AAO_CASE(512) AAO_CASE(1024) AAO_CASE(2048)
        AAO_CASE(4096) AAO_CASE(8192) AAO_CASE(16384)
#undef AAO_CASE
    default: break;
    }
    dim3 grid((n + 127) / 128, ell / 2 + 1);
    k_dft_fwd<T><<<grid, 128, 0, st>>>(r, in_scale, zprev, sigk, kap_h, n, ell,
                                       reinterpret_cast<cx<T> *>(spec), lds,
                                       reinterpret_cast<const cx<double> *>(tw));
    return hipGetLastError();
}

template <typename T>
static hipError_t inv_dispatch(const void *spec, int lds, double *z, int n, int ell,
                               const double *tw, hipStream_t st, int cfg, const double *out_scale)
{
    switch (ell) {
#define AAO_CASE(E) \
    case E: return inv_L<T, E / 2>(spec, lds, z, n, tw, st, cfg, out_scale);
        AAO_CASE(2) AAO_CASE(4) AAO_CASE(8) AAO_CASE(16) AAO_CASE(32) AAO_CASE(64)
        AAO_CASE(128) AAO_CASE(256) AAO_CASE(512) AAO_CASE(1024) AAO_CASE(2048)
        AAO_CASE(4096) AAO_CASE(8192) AAO_CASE(16384)
#undef AAO_CASE
    default: break;
    }
    dim3 grid((n + 127) / 128, ell);
    k_dft_inv<T><<<grid, 128, 0, st>>>(reinterpret_cast<const cx<T> *>(spec), lds, z, n, ell,
                                       reinterpret_cast<const cx<double> *>(tw));
    return hipGetLastError();
}

int fft_fwd_blocks(int ell, int n, bool single, int cfg)
{
    if (!fft_supported_fast(ell)) return 0;
    if (cfg >= 0 && !fft_config_ok(cfg, ell, n, single)) cfg = -1;
    const int L = ell / 2;
    const int P = cfg >= 16 ? 8 : (L < 16 ? L : 16);
    const int W = cfg >= 0 ? 1 << (cfg & 15) : default_w(L, P, n, single ? 4 : 8);
    return xcd_grid((n + W - 1) / W);
}

hipError_t launch_fft_fwd(const double *r, const double *in_scale, const double *zprev,
                          const double *sigk, double kappa, int n, int ell, void *spec, int lds,
                          bool single, const double *tw, hipStream_t st, int cfg,
                          double *norm_part)
{
    if (cfg >= 0 && !fft_config_ok(cfg, ell, n, single)) cfg = -1;
    if (norm_part && (zprev || !fft_supported_fast(ell))) return hipErrorInvalidValue;
    const double kap_h = kappa * (n + 1.0);   // kappa / h
    return single ? fwd_dispatch<float>(r, in_scale, zprev, sigk, kap_h, n, ell, spec, lds, tw, st,
                                        cfg, norm_part)
                  : fwd_dispatch<double>(r, in_scale, zprev, sigk, kap_h, n, ell, spec, lds, tw,
                                         st, cfg, norm_part);
}

hipError_t launch_fft_inv(const void *spec, int lds, bool single, double *z, int n, int ell,
                          const double *tw, hipStream_t st, int cfg, const double *out_scale)
{
    if (cfg >= 0 && !fft_config_ok(cfg, ell, n, single)) cfg = -1;
    if (out_scale && !fft_supported_fast(ell)) return hipErrorInvalidValue;
    return single ? inv_dispatch<float>(spec, lds, z, n, ell, tw, st, cfg, out_scale)
                  : inv_dispatch<double>(spec, lds, z, n, ell, tw, st, cfg, out_scale);
}

}  // namespace aao
