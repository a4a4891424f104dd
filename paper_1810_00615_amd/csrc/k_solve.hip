// Shifted complex tridiagonal solves of the circulant preconditioner apply
// (arXiv 1810.00615, eq. precon2para: the block diagonal middle factor
// I (x) A_0 + Lambda (x) A_1, one block per frequency; the paper solves each
// block with the Thomas algorithm, Sec. 3).
//
// Frequency row j of the half spectrum is the right-hand side of
//   hatA_j y = x,  hatA_j = alpha_j M + beta_j kappa K
//                = tridiag(e_j, d_j, e_j)   (complex symmetric Toeplitz),
//   alpha_j = sum_m a_m w^{jm},  beta_j = sum_m b_m w^{jm},  w = exp(-2 pi i/ell)
//   (conjugated for C^T),  d_j = alpha_j 4h/6 + beta_j kappa 2/h,
//   e_j = alpha_j h/6 - beta_j kappa/h.
//
// One workgroup per row.  The row is cut into chunks of CW contiguous unknowns,
// one chunk per thread; the last unknown of each chunk is a separator.  Each
// thread eliminates its chunk interior with the Thomas recurrence (no pivoting,
// as in the paper), which expresses the interior as y + u X_left + v X_right;
// the separators then satisfy a tridiagonal system with one equation per chunk,
// solved by parallel cyclic reduction in LDS; a last sweep recovers the
// interiors.  Because the blocks are Toeplitz, the interior elimination factors
// are the same for every chunk and are computed once per row.
#include "solve_core.h"

namespace aao {

// One workgroup per frequency row.  STAGE: the row passes through LDS so that the
// global accesses are coalesced, half a row at a time (the chunks of the first
// NT/2 threads, then the rest), so that the staging area is no larger than the
// reduced-system area it aliases.  Element i of chunk t of a half sits in slot
// i*(NT/2+PAD) + t, PAD = 1 (an odd row pitch), which spreads
// both the chunk-wise and the coalesced accesses over all banks.  Otherwise every
// thread reads and writes its own chunk directly.
// The right-hand sides are read from `in` (element type SI) and the solutions written
// to `out` (element type SO); in == out (with SI == SO) solves in place: a workgroup
// reads its whole row before it writes any of it.
// Rows: rpf rows per frequency (1 in one space dimension; ny on the unit square, where
// row (j, q) is the x-line of sine mode q in y of frequency j) at spectrum offset
// (j / rpf) lds + (j % rpf) sub.
template <typename A, typename SI, typename SO, int CW, int NTB, bool STAGE>
__global__ void __launch_bounds__(NTB)
k_shifted_solve(const cx<SI> *in, cx<SO> *out, int lds, int n, const double *__restrict__ sym,
                const cx<A> *__restrict__ ptab, int transpose, int *__restrict__ fail, int rpf,
                int sub)
{
    extern __shared__ unsigned char smraw[];
    const int NT = blockDim.x;
    cx<A> *tab = reinterpret_cast<cx<A> *>(smraw);
    cx<A> *red = tab + psolve_tab_entries(CW);
    cx<SI> *stage = reinterpret_cast<cx<SI> *>(red);
    cx<SO> *ostage = reinterpret_cast<cx<SO> *>(red);

    const int j = blockIdx.x;
    const int t = threadIdx.x;
    const int jf = j / rpf;
    const size_t roff = (size_t)jf * lds + (size_t)(j - jf * rpf) * sub;
    const cx<SI> *row = in + roff;
    cx<SO> *orow = out + roff;

    const int P = (n + CW - 1) / CW;
    const int a0 = t * CW;
    const int len = (t < P) ? min(CW, n - a0) : 0;

    // The row's symbol and partition table are loaded before its data, so that their
    // latency is not added after the data arrive; the table goes to LDS while the
    // data loads are in flight.
    const double *sj = sym + ((size_t)j * 2 + (transpose ? 1 : 0)) * 4;
    const cx<A> d = {A(sj[0]), A(sj[1])};
    const cx<A> e = {A(sj[2]), A(sj[3])};
    const cx<A> *rtab = ptab + ((size_t)j * 2 + (transpose ? 1 : 0)) * psolve_tab_entries(CW);
    const bool tab_lane = t < psolve_tab_entries(CW);
    const cx<A> tv = tab_lane ? rtab[t] : cx<A>{A(0), A(0)};
    constexpr int PAD = 1;
    constexpr int OPAD = 1;
    const int NH = NT / 2;                       // threads per staged half
    const int NTP = NH + PAD;
    const int ONTP = NH + OPAD;
    const int H = NH * CW;                       // unknowns per staged half
    const int mine = t / NH;                     // the half holding this thread's chunk
    const int tl = t - mine * NH;
    cx<A> y[CW];
#pragma unroll
    for (int i = 0; i < CW; ++i) y[i] = {A(0), A(0)};
    if (STAGE) {
        // H / NT = CW / 2 elements per thread and half, loaded together (unconditional
        // at a clamped index; a guarded load per element would be waited for in turn).
        // The second half's loads are issued as soon as the first half sits in LDS (into
        // the same registers), so they are in flight while the first half is read.
        constexpr int KH = CW >= 2 ? CW / 2 : 1;
        SI lx[KH], ly[KH];   // separate parts: a whole-struct array would live in scratch
        auto load_half = [&](int q0) {
#pragma unroll
            for (int k = 0; k < KH; ++k) {
                const cx<SI> v = row[min(q0 + t + k * NT, n - 1)];
                lx[k] = v.x;
                ly[k] = v.y;
            }
        };
        auto stage_half = [&](int q0) {
            const int q1 = min(n, q0 + H);
#pragma unroll
            for (int k = 0; k < KH; ++k) {
                const int q = q0 + t + k * NT;
                if (q < q1) {
                    const int ql = q - q0;
                    stage[(ql % CW) * NTP + ql / CW] = {lx[k], ly[k]};
                }
            }
        };
        auto read_half = [&]() {
#pragma unroll
            for (int i = 0; i < CW; ++i)
                if (i < len) {
                    const cx<SI> v = stage[i * NTP + tl];
                    y[i] = {A(v.x), A(v.y)};
                }
        };
        load_half(0);
        if (tab_lane) tab[t] = tv;               // (the table does not alias the staging)
        stage_half(0);
        load_half(H);
        __syncthreads();
        if (mine == 0) read_half();
        __syncthreads();                         // the first half has been read
        stage_half(H);
        __syncthreads();
        if (mine == 1) read_half();
        // partition_solve's first barrier precedes its first write to the area
    } else {
#pragma unroll
        for (int i = 0; i < CW; ++i) {
            const cx<SI> v = row[min(a0 + i, n - 1)];   // unconditional: all in flight
            if (i < len) y[i] = {A(v.x), A(v.y)};
        }
        if (tab_lane) tab[t] = tv;
    }

    // the table was written to LDS above; partition_solve's first barrier orders it
    const bool bad = partition_solve<A, CW, kTabReady>(y, n, d, e, tab, red);
    if (STAGE) {
        for (int half = 0; half < 2; ++half) {
            const int q0 = half * H;
            const int q1 = min(n, q0 + H);
            if (half == 1) __syncthreads();      // the first half has been stored
            if (mine == half) {
#pragma unroll
                for (int i = 0; i < CW; ++i)
                    if (i < len) ostage[i * ONTP + tl] = {SO(y[i].x), SO(y[i].y)};
            }
            __syncthreads();
            for (int q = q0 + t; q < q1; q += NT) {
                const int ql = q - q0;
                orow[q] = ostage[(ql % CW) * ONTP + ql / CW];
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < CW; ++i)
            if (i < len) orow[a0 + i] = {SO(y[i].x), SO(y[i].y)};
    }
    if (bad && fail) atomicOr(fail, 1);
}

// Launch configurations {chunk CW, threads NT}; configuration k < kNumSolveCfg
// reads chunks directly, k + kNumSolveCfg stages the row through LDS half a row at
// a time.  A row of n unknowns needs n <= CW * NT.
static const int kSolveCfg[][2] = {{1, 256}, {2, 256}, {4, 256}, {8, 256}, {8, 512},
                                   {8, 1024}, {16, 128}, {16, 256}, {16, 512}, {16, 1024},
                                   {32, 128}, {32, 256}, {4, 64}, {8, 64}, {16, 64},
                                   {4, 128}, {8, 128}};
constexpr int kNumSolveCfg = sizeof(kSolveCfg) / sizeof(kSolveCfg[0]);

int solve_num_configs() { return 2 * kNumSolveCfg; }

// LDS bytes of a configuration, for 16-byte complex elements (the largest case)
static size_t solve_lds_bytes(int cw, int nt, bool stage)
{
    const size_t red = 16 * (size_t)psolve_lds_entries(cw, nt);
    const size_t stg = 16 * ((size_t)psolve_tab_entries(cw) + (size_t)cw * (nt / 2 + 2));
    return stage && stg > red ? stg : red;
}

bool solve_config_ok(int cfg, int n)
{
    if (cfg < 0 || cfg >= 2 * kNumSolveCfg) return false;
    const int k = cfg % kNumSolveCfg;
    return n <= kSolveCfg[k][0] * kSolveCfg[k][1] &&
           solve_lds_bytes(kSolveCfg[k][0], kSolveCfg[k][1], cfg >= kNumSolveCfg) <= 160 * 1024;
}

void solve_config_shape(int cfg, int *cw, int *nt, int *stage)
{
    const int k = cfg % kNumSolveCfg;
    *cw = kSolveCfg[k][0];
    *nt = kSolveCfg[k][1];
    *stage = cfg >= kNumSolveCfg;
}

// default: the half-staged configuration with the smallest chunk (then the fewest
// threads) that covers n with at most 512 threads; beyond that the widest
// configuration that fits
int solve_default_config(int n)
{
    int best = -1;
    for (int k = 0; k < kNumSolveCfg; ++k) {
        const int cw = kSolveCfg[k][0], nt = kSolveCfg[k][1];
        if (nt > 512 || !solve_config_ok(k + kNumSolveCfg, n)) continue;
        if (best < 0 || cw < kSolveCfg[best][0] ||
            (cw == kSolveCfg[best][0] && nt < kSolveCfg[best][1]))
            best = k;
    }
    if (best >= 0) return best + kNumSolveCfg;
    for (int c = 2 * kNumSolveCfg - 1; c >= 0; --c)
        if (solve_config_ok(c, n)) return c;
    return -1;
}

template <typename S>
static constexpr size_t stage_bytes(int cw, int nt)
{
    return sizeof(cx<S>) * (size_t)cw * (nt / 2 + 1);
}

template <typename A, typename SI, typename SO, int CW, int NT, bool STAGE>
static hipError_t solve_go(const void *in, void *out, int lds, int n, int ell, const double *sym,
                           const void *ptab, int transpose, int *fail, hipStream_t st, int rpf,
                           int sub)
{
    size_t smem = sizeof(cx<A>) * psolve_lds_entries(CW, NT);
    if (STAGE) {
        const size_t so = stage_bytes<SI>(CW, NT) > stage_bytes<SO>(CW, NT)
                              ? stage_bytes<SI>(CW, NT)
                              : stage_bytes<SO>(CW, NT);
        const size_t stg = sizeof(cx<A>) * psolve_tab_entries(CW) + so;
        if (stg > smem) smem = stg;
    }
    auto kern = k_shifted_solve<A, SI, SO, CW, NT, STAGE>;
    if (smem > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    kern<<<(ell / 2 + 1) * rpf, NT, smem, st>>>(reinterpret_cast<const cx<SI> *>(in),
                                                reinterpret_cast<cx<SO> *>(out), lds, n, sym,
                                                reinterpret_cast<const cx<A> *>(ptab), transpose,
                                                fail, rpf, sub);
    return hipGetLastError();
}

template <typename A, typename SI, typename SO>
static hipError_t solve_disp(int cfg, const void *in, void *out, int lds, int n, int ell,
                             const double *sym, const void *ptab, int transpose, int *fail,
                             hipStream_t st, int rpf, int sub)
{
    const bool stage = cfg >= kNumSolveCfg;
#define AAO_SCFG(I, CW, NT)                                                                    \
    case I:                                                                                    \
        return stage ? solve_go<A, SI, SO, CW, NT, true>(in, out, lds, n, ell, sym, ptab,        \
                                                         transpose, fail, st, rpf, sub)        \
                     : solve_go<A, SI, SO, CW, NT, false>(in, out, lds, n, ell, sym, ptab,       \
                                                          transpose, fail, st, rpf, sub);
    switch (cfg % kNumSolveCfg) {
        AAO_SCFG(0, 1, 256)
        AAO_SCFG(1, 2, 256)
        AAO_SCFG(2, 4, 256)
        AAO_SCFG(3, 8, 256)
        AAO_SCFG(4, 8, 512)
        AAO_SCFG(5, 8, 1024)
        AAO_SCFG(6, 16, 128)
        AAO_SCFG(7, 16, 256)
        AAO_SCFG(8, 16, 512)
        AAO_SCFG(9, 16, 1024)
        AAO_SCFG(10, 32, 128)
        AAO_SCFG(11, 32, 256)
        AAO_SCFG(12, 4, 64)
        AAO_SCFG(13, 8, 64)
        AAO_SCFG(14, 16, 64)
        AAO_SCFG(15, 4, 128)
        AAO_SCFG(16, 8, 128)
    default: return hipErrorInvalidValue;
    }
#undef AAO_SCFG
}

// ------------------------------------------------- checkpoint recomputation
// Heat trajectory between checkpoints, for the kappa gradient.  Segment s covers
// time levels [s*stride, min((s+1)*stride, ell)) (0-based rows); it starts from
// u0 (s = 0) or the stored row s*stride - 1 and takes implicit Euler steps
// (M + tau_k kappa K) u_k = M u_{k-1} (eq. timestepproblem1 read as M + tau K), each
// step a partition solve by the whole workgroup.  While stepping it accumulates
// sum_k tau_k lam_k . (K u_k), the term of dL/dkappa that needs U.
template <int CW>
__global__ void __launch_bounds__(256)
k_heat_segments(const double *__restrict__ u0, const double *__restrict__ Uck, int stride,
                const double *__restrict__ lam, int n, int ell, double tau, double kappa,
                const double *__restrict__ tau_k, double *__restrict__ part,
                double *__restrict__ Uout, int *__restrict__ fail)
{
    extern __shared__ unsigned char smraw[];
    const int NT = blockDim.x;
    const int t = threadIdx.x;
    cx<double> *tab = reinterpret_cast<cx<double> *>(smraw);
    cx<double> *red = tab + psolve_tab_entries(CW);                         // 6*NT entries
    double *edge = reinterpret_cast<double *>(red + 6 * NT); // first/last value of every chunk
    __shared__ double wsum[16];

    const int seg = blockIdx.x;
    const int kb = seg * stride;
    const int ke = min(kb + stride, ell);
    const double *start = seg == 0 ? u0 : Uck + (size_t)(seg - 1) * n;
    const double h = 1.0 / (n + 1.0);
    const int a0 = t * CW;
    const int P = (n + CW - 1) / CW;
    const int len = (t < P) ? min(CW, n - a0) : 0;

    double u[CW];
#pragma unroll
    for (int i = 0; i < CW; ++i) u[i] = (i < len) ? start[a0 + i] : 0.0;

    // neighbours of the chunk ends through LDS: (left of first, right of last)
    auto halo = [&](double &left, double &right) {
        double first = 0.0, last = 0.0;
#pragma unroll
        for (int i = 0; i < CW; ++i) {
            if (i == 0) first = u[i];
            if (i == len - 1) last = u[i];
        }
        if (t < P) {
            edge[2 * t] = first;
            edge[2 * t + 1] = last;
        }
        __syncthreads();
        left = (t > 0 && t < P) ? edge[2 * (t - 1) + 1] : 0.0;
        right = (t + 1 < P) ? edge[2 * (t + 1)] : 0.0;
        __syncthreads();
    };

    double acc = 0.0;
    bool bad = false;
    for (int k = kb; k < ke; ++k) {
        const double tk = tau_k ? tau_k[k] : tau;
        // right-hand side M u_{k-1}
        double left, right;
        halo(left, right);
        cx<double> y[CW];
#pragma unroll
        for (int i = 0; i < CW; ++i) {
            const double ul = (i == 0) ? left : u[i > 0 ? i - 1 : 0];
            const double ur = (i == len - 1) ? right : u[i < CW - 1 ? i + 1 : CW - 1];
            y[i] = {(i < len) ? (h / 6.0) * (ul + 4.0 * u[i] + ur) : 0.0, 0.0};
        }
        const cx<double> d = {4.0 * h / 6.0 + tk * kappa * 2.0 / h, 0.0};
        const cx<double> e = {h / 6.0 - tk * kappa / h, 0.0};
        bad |= partition_solve<double, CW>(y, n, d, e, tab, red);
#pragma unroll
        for (int i = 0; i < CW; ++i) u[i] = (i < len) ? y[i].x : 0.0;
        if (Uout) {
#pragma unroll
            for (int i = 0; i < CW; ++i)
                if (i < len) Uout[(size_t)k * n + a0 + i] = u[i];
        }
        // tau_k lam_k . K u_k
        halo(left, right);
        const double *lk = lam + (size_t)k * n;
#pragma unroll
        for (int i = 0; i < CW; ++i) {
            if (i < len) {
                const double ul = (i == 0) ? left : u[i > 0 ? i - 1 : 0];
                const double ur = (i == len - 1) ? right : u[i < CW - 1 ? i + 1 : CW - 1];
                acc += tk * lk[a0 + i] * (2.0 * u[i] - ul - ur) / h;
            }
        }
    }
    // block sum in a fixed order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((t & 63) == 0) wsum[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
        double sacc = 0.0;
        for (int w = 0; w < NT / 64; ++w) sacc += wsum[w];
        part[seg] = sacc;
    }
    if (bad && fail) atomicOr(fail, 1);
}

hipError_t launch_heat_segments(const double *u0, const double *Uck, int stride, const double *lam,
                                int n, int ell, double tau, double kappa, const double *tau_k,
                                double *part, double *Uout, int *fail, hipStream_t st)
{
    const int NT = 256;
    int cw = 1;
    while (cw * NT < n) cw *= 2;
    if (cw > 16) return hipErrorInvalidValue;
    const int nseg = (ell + stride - 1) / stride;
    const size_t smem = sizeof(cx<double>) * psolve_lds_entries(cw, NT) + sizeof(double) * 2 * NT;
    auto go = [&](auto kern) -> hipError_t {
        if (smem > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void *)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)smem);
            if (e != hipSuccess) return e;
        }
        kern<<<nseg, NT, smem, st>>>(u0, Uck, stride, lam, n, ell, tau, kappa, tau_k, part, Uout,
                                     fail);
        return hipGetLastError();
    };
    switch (cw) {
    case 1: return go(k_heat_segments<1>);
    case 2: return go(k_heat_segments<2>);
    case 4: return go(k_heat_segments<4>);
    case 8: return go(k_heat_segments<8>);
    default: return go(k_heat_segments<16>);
    }
}

// d_j, e_j of every half-spectrum row, for the symbol (tr = 0) and its conjugate
// (tr = 1): sym[(2 j + tr) * 4 + {0, 1, 2, 3}] = Re d, Im d, Re e, Im e with
//   alpha_j = sum_m a_m w^{jm},  beta_j = sum_m b_m w^{jm},  w = exp(-+2 pi i/ell),
//   m over the Toeplitz offsets -up..s (BD4: (1 - w^j)^2 (2 - w^j); central
//   differences: w^{-j} - 2 + w^j = -4 sin^2(pi j / ell), real),
//   d_j = alpha_j 4h/6 + beta_j kappa 2/h,  e_j = alpha_j h/6 - beta_j kappa/h.
// On the unit square (ny > 0; Q1 blocks alpha My (x) Mx + beta kappa (Ky (x) Mx +
// My (x) Kx)) the sine transform in y leaves, for mode q = 1..ny of row (j, q - 1),
// the x-tridiagonal A Mx + B Kx with A = alpha my_q + beta kappa ky_q, B = beta kappa my_q,
//   my_q = hy/6 (4 + 2 cos(pi q/(ny+1))),  ky_q = 4 sin^2(pi q/(2(ny+1))) / hy,
// so d = A 4h/6 + B 2/h, e = A h/6 - B/h with h = 1/(n+1) the x spacing.
__global__ void k_symbols(double *__restrict__ sym, int n, int ell, Scheme sc, double kappa,
                          int ny)
{
    const int rpf = ny > 0 ? ny : 1;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (ell / 2 + 1) * rpf) return;
    const int j = r / rpf;
    const double h = 1.0 / (n + 1.0);
    double my = 1.0, ky = 0.0;
    if (ny > 0) {
        const int q = r - j * rpf + 1;
        const double hy = 1.0 / (ny + 1.0);
        const double sh = sinpi((double)q / (2.0 * (ny + 1.0)));
        my = hy / 6.0 * (4.0 + 2.0 * cospi((double)q / (ny + 1.0)));
        ky = 4.0 * sh * sh / hy;
    }
    for (int tr = 0; tr < 2; ++tr) {
        double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
        for (int m = -sc.up; m <= sc.s; ++m) {
            // the Toeplitz blocks (start-up rows are not part of the circulant)
            const double am = m < 0 ? sc.au : sc.a[m], bm = m < 0 ? sc.bu : sc.b[m];
            const long long p = (((long long)j * m) % ell + ell) % ell;
            double sn, cs;
            sincospi((tr ? 2.0 : -2.0) * (double)p / (double)ell, &sn, &cs);
            ar += am * cs;
            ai += am * sn;
            br += bm * cs;
            bi += bm * sn;
        }
        // A = alpha my + beta kappa ky, B = beta kappa my
        const double Ar = ar * my + br * kappa * ky, Ai = ai * my + bi * kappa * ky;
        const double Br = br * kappa * my, Bi = bi * kappa * my;
        double *o = sym + ((size_t)r * 2 + tr) * 4;
        o[0] = Ar * (4.0 * h / 6.0) + Br * (2.0 / h);
        o[1] = Ai * (4.0 * h / 6.0) + Bi * (2.0 / h);
        o[2] = Ar * (h / 6.0) - Br / h;
        o[3] = Ai * (h / 6.0) - Bi / h;
    }
}

hipError_t launch_symbols(double *sym, int n, int ell, Scheme sc, double kappa, hipStream_t st,
                          int ny)
{
    const int rows = (ell / 2 + 1) * (ny > 0 ? ny : 1);
    k_symbols<<<(rows + 255) / 256, 256, 0, st>>>(sym, n, ell, sc, kappa, ny);
    return hipGetLastError();
}

// Partition tables of every row and orientation for chunk width CW (build_tab):
// out[((2 j + tr) * psolve_tab_entries(CW) + i], one thread per (row, orientation).
template <typename A, int CW>
__global__ void k_ptab(const double *__restrict__ sym, int rows, int n, cx<A> *__restrict__ out)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= 2 * rows) return;
    const double *sj = sym + (size_t)id * 4;
    const cx<A> d = {A(sj[0]), A(sj[1])};
    const cx<A> e = {A(sj[2]), A(sj[3])};
    const int P = (n + CW - 1) / CW;
    build_tab<A, CW>(d, e, n - (P - 1) * CW - 1, out + (size_t)id * psolve_tab_entries(CW));
}

size_t solve_table_bytes(int ell, int rpf)
{
    return sizeof(cx<double>) * 2 * (size_t)(ell / 2 + 1) * (size_t)rpf * psolve_tab_entries(32);
}

int solve_effective_config(int cfg, int n)
{
    return solve_config_ok(cfg, n) ? cfg : solve_default_config(n);
}

template <typename A>
static hipError_t ptab_disp(int cw, const double *sym, int n, int ell, void *out, hipStream_t st,
                            int rpf)
{
    const int rows = (ell / 2 + 1) * rpf;
    const int grid = (2 * rows + 255) / 256;
    cx<A> *o = reinterpret_cast<cx<A> *>(out);
    switch (cw) {
    case 1: k_ptab<A, 1><<<grid, 256, 0, st>>>(sym, rows, n, o); break;
    case 2: k_ptab<A, 2><<<grid, 256, 0, st>>>(sym, rows, n, o); break;
    case 4: k_ptab<A, 4><<<grid, 256, 0, st>>>(sym, rows, n, o); break;
    case 8: k_ptab<A, 8><<<grid, 256, 0, st>>>(sym, rows, n, o); break;
    case 16: k_ptab<A, 16><<<grid, 256, 0, st>>>(sym, rows, n, o); break;
    case 32: k_ptab<A, 32><<<grid, 256, 0, st>>>(sym, rows, n, o); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_solve_tables(const double *sym, int n, int ell, int cfg, bool single_arith,
                               void *out, hipStream_t st, int rpf)
{
    cfg = solve_effective_config(cfg, n);
    if (cfg < 0 || rpf < 1) return hipErrorInvalidValue;
    int cw, nt, stage;
    solve_config_shape(cfg, &cw, &nt, &stage);
    return single_arith ? ptab_disp<float>(cw, sym, n, ell, out, st, rpf)
                        : ptab_disp<double>(cw, sym, n, ell, out, st, rpf);
}

hipError_t launch_shifted_solve(const void *in, void *out, int lds, bool single_in,
                                bool single_out, bool single_arith, int n, int ell,
                                const double *sym, const void *ptab, int transpose,
                                int *fail_flag, hipStream_t st, int cfg, int rpf, int sub)
{
    cfg = solve_effective_config(cfg, n);
    if (cfg < 0 || !ptab || rpf < 1) return hipErrorInvalidValue;
    if (in == out && single_in != single_out) return hipErrorInvalidValue;
    if (single_arith) {
        if (!single_in || !single_out) return hipErrorInvalidValue;
        return solve_disp<float, float, float>(cfg, in, out, lds, n, ell, sym, ptab, transpose,
                                               fail_flag, st, rpf, sub);
    }
    if (!single_in && !single_out)
        return solve_disp<double, double, double>(cfg, in, out, lds, n, ell, sym, ptab,
                                                  transpose, fail_flag, st, rpf, sub);
    if (single_in && single_out)
        return solve_disp<double, float, float>(cfg, in, out, lds, n, ell, sym, ptab, transpose,
                                                fail_flag, st, rpf, sub);
    if (single_in)
        return solve_disp<double, float, double>(cfg, in, out, lds, n, ell, sym, ptab,
                                                 transpose, fail_flag, st, rpf, sub);
    return hipErrorInvalidValue;
}

}  // namespace aao
