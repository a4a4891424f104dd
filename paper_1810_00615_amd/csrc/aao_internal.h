// Internal declarations shared by the HIP translation units of libaao.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aao {

// ----------------------------------------------------------------- complex
template <typename T> struct cx { T x, y; };

template <typename T> __host__ __device__ inline cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a) { return {-a.x, -a.y}; }
template <typename T> __host__ __device__ inline cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
__host__ __device__ inline double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ inline float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// a + b c and a - b c, each component two fused multiply-adds
template <typename T> __host__ __device__ inline cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
    return {ffma(b.x, c.x, ffma(-b.y, c.y, a.x)), ffma(b.x, c.y, ffma(b.y, c.x, a.y))};
}
template <typename T> __host__ __device__ inline cx<T> cfms(cx<T> a, cx<T> b, cx<T> c) {
    return {ffma(-b.x, c.x, ffma(b.y, c.y, a.x)), ffma(-b.x, c.y, ffma(-b.y, c.x, a.y))};
}
// i * a
template <typename T> __host__ __device__ inline cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }
// 1 / a (scaled to avoid overflow of |a|^2 for the magnitudes seen here)
template <typename T> __host__ __device__ inline cx<T> recip(cx<T> a) {
    T d = a.x * a.x + a.y * a.y;
    T inv = T(1) / d;
    return {a.x * inv, -a.y * inv};
}

// ------------------------------------------------------------- scheme data
// The block in row k, column k - m of the monolithic matrix is a_m M + b_m kappa K
// for the Toeplitz rows, m = 0..s (s <= 3); with up = 1 also one block above the
// diagonal (m = -1): au M + bu kappa K; the first nst rows (nst <= 2) are start-up
// rows with their own lower blocks sa[k][m] M + sb[k][m] kappa K (zero pairs absent).
// The circulant preconditioner wraps the Toeplitz blocks (m = -up..s).
struct Scheme {
    int id;            // AAO_HEAT_IE, AAO_WAVE_BD2, ...
    int s;
    double a[4];
    double b[4];
    int up;
    double au, bu;
    int nst;
    double sa[2][4], sb[2][4];
};
// schemes whose matvec is not the plain lower-triangular Toeplitz one
__host__ __device__ inline bool scheme_generic(const Scheme &sc) { return sc.up || sc.nst > 0; }
// coefficients (cm, cb) of the block in row `row`, offset m (cm M + cb kappa K); false
// if that block is zero (row and column bounds are the caller's)
__host__ __device__ inline bool scheme_block(const Scheme &sc, int row, int m, double &cm,
                                             double &cb)
{
    if (m < 0) {
        if (m < -1 || !sc.up) return false;
        cm = sc.au;
        cb = sc.bu;
    } else {
        if (m > sc.s) return false;
        const bool st = row < sc.nst;
        cm = st ? sc.sa[row][m] : sc.a[m];
        cb = st ? sc.sb[row][m] : sc.b[m];
    }
    return cm != 0.0 || cb != 0.0;
}

// Tuned launch shapes, cached per process and in the aao_set_tune_cache file, keyed by
// (device, kind, precision, n, ell); a batch stores its shapes under kinds >= 100 with
// n = the member count and ell = a hash of the member sizes.
bool tune_cache_get(int device, int kind, int prec, int64_t n, int64_t ell, int *code);
void tune_cache_put(int device, int kind, int prec, int64_t n, int64_t ell, int code, double us);

// Coefficients of a scheme constant of aao.h (AAO_HEAT_IE, ...) for step tau; false
// for an unknown scheme.
bool make_scheme(int scheme, double tau, Scheme *out);

// ------------------------------------------------------------ launchers
// All launchers enqueue on `st` and return hipError_t of the launch.

// Twiddle table w_len^p = exp(-2 pi i p / len), p in [0, count).
hipError_t launch_twiddles(double *tw, int len, int count, hipStream_t st);

// Forward half-spectrum transform along time of the ell x n real array
// src = r - E zprev (E term only if zprev != nullptr):
// spec rows j = 0..ell/2 (complex, leading dimension lds, element type
// float2/double2 according to `single`).
// in_scale (device scalar or nullptr) multiplies r.
// cfg: launch shape (16 v + log2 W, see fft_configs), negative = default.
// norm_part (power-of-two ell, no zprev): one partial of ||r||^2 (r unscaled) per
// workgroup, fft_fwd_blocks() of them.
hipError_t launch_fft_fwd(const double *r, const double *in_scale, const double *zprev,
                          const double *sigk, double kappa, int n, int ell, void *spec, int lds,
                          bool single, const double *tw, hipStream_t st, int cfg = -1,
                          double *norm_part = nullptr);
int fft_fwd_blocks(int ell, int n, bool single, int cfg);
// Inverse of the above: z (ell x n real) from the half spectrum, times *out_scale
// (device scalar, power-of-two ell) if given.
hipError_t launch_fft_inv(const void *spec, int lds, bool single, double *z, int n, int ell,
                          const double *tw, hipStream_t st, int cfg = -1,
                          const double *out_scale = nullptr);
// Admissible launch shapes of the power-of-two transforms for (ell, n, element
// type): writes up to cap of them to out, returns how many there are (0 when ell
// is not a supported power of two).
int fft_configs(int ell, int n, bool single, int *out, int cap);
bool fft_config_ok(int cfg, int ell, int n, bool single);
// Shifted solves (alpha_j M + beta_j kappa K) Y_j = X_j for every half-spectrum row
// j: X from `in` (float2 rows if single_in, else double2), Y to `out` (float2 if
// single_out); in == out solves in place (same element type).  `single_arith`
// selects single-precision arithmetic (single in and out only).  sym: the per-row
// table of launch_symbols; ptab: the partition tables of launch_solve_tables for the
// same configuration and arithmetic.  cfg selects the launch shape (chunk, threads,
// LDS staging) among solve_num_configs(); a value that is out of range or does not
// cover n selects solve_default_config(n).
// rpf > 1 (unit square, rpf = ny): every frequency has rpf rows of n unknowns, row q of
// frequency j at offset j lds + q sub of the spectrum.
hipError_t launch_shifted_solve(const void *in, void *out, int lds, bool single_in,
                                bool single_out, bool single_arith, int n, int ell,
                                const double *sym, const void *ptab, int transpose,
                                int *fail_flag, hipStream_t st, int cfg = -1, int rpf = 1,
                                int sub = 0);
// Per-row symbol table, (ell/2 + 1) rpf rows x 2 orientations x (d, e) complex = 8
// doubles a row; ny > 0 selects the Q1 blocks of the unit square (rpf = ny, n = nx).
hipError_t launch_symbols(double *sym, int n, int ell, Scheme sc, double kappa, hipStream_t st,
                          int ny = 0);
// Partition tables (interior elimination factors and response end values) of every
// row and orientation for the chunk width of configuration cfg, in the solve's
// arithmetic; out holds solve_table_bytes(ell, rpf).
hipError_t launch_solve_tables(const double *sym, int n, int ell, int cfg, bool single_arith,
                               void *out, hipStream_t st, int rpf = 1);
size_t solve_table_bytes(int ell, int rpf = 1);
int solve_effective_config(int cfg, int n);
int solve_num_configs();
bool solve_config_ok(int cfg, int n);
void solve_config_shape(int cfg, int *cw, int *nt, int *stage);
int solve_default_config(int n);
bool fft_supported_fast(int ell);
// Heat trajectory recomputed from checkpoints (every `stride` rows) while
// accumulating part[seg] = sum_k tau_k lam_k . K u_k over each segment.
hipError_t launch_heat_segments(const double *u0, const double *Uck, int stride, const double *lam,
                                int n, int ell, double tau, double kappa, const double *tau_k,
                                double *part, double *Uout, int *fail, hipStream_t st);

// y = A x (or A^T x); with tau_k != nullptr the variable-step matrix B.
// If bsub != nullptr computes y = bsub - A x.  With nv > 0 the launch also writes the
// block partials of V_q . y (q < nv) and of y . y (value nv); nv == 1 with
// V->p[0] == y selects only the partials of y . y (value 0).  y may be null (nothing
// stored; only with the self-norm).
struct VecList;
hipError_t launch_matvec(const double *x, double *y, const double *bsub, int n, int ell,
                         Scheme sc, double kappa, const double *tau_k, int transpose,
                         hipStream_t st, int cfg = -1, const VecList *V = nullptr, int nv = 0,
                         double *part = nullptr, int ldp = 0);
// x given as a combination sum_q c[q] z[q] (q < 4) and written to xout by the matvec
struct MatvecComb {
    const double *z[4];
    double c[4];
    double *xout;
};
// The residual check of a solution update in one launch: x = sum_{q<nz} c_q z_q is
// formed on the fly, written to cb.xout, and the block partials of |bsub - A x|^2 go to
// part (one value).  Only for DPP launch shapes and nz <= 4 (matvec_comb_ok).
bool matvec_comb_ok(int cfg, int nz);
hipError_t launch_matvec_comb(const MatvecComb &cb, int nz, const double *bsub, int n, int ell,
                              Scheme sc, double kappa, const double *tau_k, int transpose,
                              hipStream_t st, int cfg, double *part, int ldp);
// matvec launch shapes: code = 3 v + r (R = 4 << r rows per thread, v = 1: DPP lane moves)
int matvec_num_configs();
int matvec_default_config();
// number of workgroups (= partials per dot value) of a matvec launch
int matvec_blocks(int n, int ell, int cfg);
hipError_t launch_project_sine(double *u0, int n, int J, const int *modes, const double *amps,
                               hipStream_t st);
hipError_t launch_build_rhs(double *b, const double *u0, const double *v0, int n, int ell,
                            Scheme sc, double kappa, double tau, hipStream_t st);

// ------------------------------------------------------- Krylov helpers
// Up to kMaxVecs device vectors / coefficients, passed to kernels by value.
constexpr int kMaxVecs = 64;
struct VecList {
    const double *p[kMaxVecs];
};
struct CoefList {
    double v[kMaxVecs];
};
// Partial dot products, value-major: part[i * ldp + blk] = sum over block blk's
// slice of V_i . w, i < nv (dot_blocks(N) blocks, ldp >= that count).
int dot_blocks(size_t N);
hipError_t launch_multidot(const VecList &V, int nv, const double *w, size_t N, double *part,
                           int ldp, hipStream_t st);
// w' = w - sum_i V_i h_i (h device) and the partials of V_i . w' (i < nv).  w is
// not modified.
hipError_t launch_update_dot(const VecList &V, int nv, const double *w, const double *h,
                             size_t N, double *part, int ldp, hipStream_t st);
// out = w - sum_i V_i h_i and the partials of out.out (value 0).
hipError_t launch_update_norm(const VecList &V, int nv, const double *w, const double *h,
                              double *out, size_t N, double *part, int ldp, hipStream_t st);
// sums[i] = sum_blk part[i * ldp + blk] in fixed order, i < cnt
hipError_t launch_reduce_parts(const double *part, int nblk, int ldp, int cnt, double *sums,
                               hipStream_t st);
// x = (accumulate ? x : 0) + sum_i Z_i y_i
hipError_t launch_multi_axpy(const VecList &Z, int nz, const CoefList &y, double *x, size_t N,
                             bool accumulate, hipStream_t st);
// Arnoldi update with delayed re-orthogonalisation, step j (nv = j + 1 basis vectors
// S_0..S_j, S_j the pending vector p):
//   v_j = sum_i cv_i S_i  (written to vout unless vout is null),
//   w1  = w - sum_i cw_i S_i  (written to wout),
// and the partials of S_i . w1 (i < j), v_j . w1 (value j) and w1 . w1 (value nv).
hipError_t launch_arnoldi_update(const VecList &S, int nv, const double *w, const double *cv,
                                 const double *cw, double *vout, double *wout, size_t N,
                                 double *part, int ldp, hipStream_t st);
// Slots of the mapped host buffer written by k_reduce_small.
constexpr int kHostBeta = kMaxVecs;       // residual norm
constexpr int kHostBB = kMaxVecs + 1;     // b.b
constexpr int kHostFail = kMaxVecs + 2;   // shifted-solve breakdown flag (0 / 1)
constexpr int kHostSeq = kMaxVecs + 3;    // sequence number of the last reduction
constexpr int kHostWW = 2 * kMaxVecs + 4; // w . w of the step's matvec
constexpr int kHostA = kMaxVecs + 4;      // re-orthogonalisation coefficients (kMaxVecs)
constexpr int kHostSlots = 2 * kMaxVecs + 8;
struct SmallArgs {
    int mode, nv;
    double *h1, *h2, *c, *vs;   // device scalars (kMaxVecs + 1 each)
    double *host;               // device view of the mapped host buffer
    const int *fail;
    double *a, *cv, *cw;        // delayed re-orthogonalisation scalars (kMaxVecs + 1 each)
    double seq;                 // written to host[kHostSeq] after every other result
};
// Fused fixed-order reduction of one Krylov step's partials and its scalar update
// (modes documented at the kernel).
hipError_t launch_reduce_small(const double *part, int nblk, int ldp, const SmallArgs &a,
                               hipStream_t st);
// out = w * (*scale)
hipError_t launch_scale(const double *w, const double *scale, double *out, size_t N,
                        hipStream_t st);
// out = a * w (host scalar a)
hipError_t launch_scale_h(const double *w, double a, double *out, size_t N, hipStream_t st);
hipError_t launch_fill(double *x, double v, size_t N, hipStream_t st);
// out = s r - blockdiag(sigma_k kappa K) z, s = *scale (nullptr: 1); ell x n vectors
hipError_t launch_neumann_rhs(const double *r, const double *scale, const double *z,
                              const double *sigk, double kappa, int n, int ell, double *out,
                              hipStream_t st);

// Gradient reduction helpers
// partial sums of sum_k sum_m c_m^{(k)} lam_k . K u_{k-m} (negated later)
hipError_t launch_grad_kappa_parts(const double *U, const double *lam, int n, int ell,
                                   Scheme sc, const double *tau_k, double *part, int nblk,
                                   hipStream_t st);
// y = (cm M + ck K) x for one n-vector, plus optional y += (cm2 M + ck2 K) x2 and
// y += (cm3 M + ck3 K) x3
hipError_t launch_mk(const double *x, double cm, double ck, const double *x2, double cm2,
                     double ck2, double *y, int n, hipStream_t st, const double *x3 = nullptr,
                     double cm3 = 0.0, double ck3 = 0.0);
hipError_t launch_dot1_parts(const double *a, const double *b, size_t N, double *part,
                             hipStream_t st);

// ------------------------------------------------- unit square (Q1 elements)
// Vectors of one time level are ny x nx, x fastest; ell levels follow each other.
// Orthonormal sine transform along y of every level (its own inverse); in == out
// allowed.  Needs ny + 1 a power of two, ny <= 2047; tw the twiddle table of length
// 2 (ny + 1) (launch_twiddles): the length-(ny + 1) transform takes every other entry.
bool dst_y_supported(int ny);
hipError_t launch_dst_y(const double *in, double *out, int nx, int ny, int ell, const double *tw,
                        hipStream_t st);
// y = A x (A^T x with transpose), y = bsub - A x if bsub, for the Q1 blocks
// a_m M2 + b_m kappa K2 (M2 = My (x) Mx, K2 = Ky (x) Mx + My (x) Kx).  With nv > 0 the
// launch also leaves the block partials of V_q . y (q < nv) and of y . y (value nv);
// nv == 1 with V->p[0] == y only those of y . y (value 0); y may then be null.
// matvec2d_blocks(..., true) partials per value.  With nv > matvec2d_dot_walk() the
// dots past the first ones read y back, so y must not be null.  With hat the vectors
// are in sine coordinates along y (S_y A S_y: x-stencils per sine mode); the forms with
// dot products (GMRES) exist in those coordinates only.
hipError_t launch_matvec2d(const double *x, double *y, const double *bsub, int nx, int ny,
                           int ell, Scheme sc, double kappa, int transpose, hipStream_t st,
                           const VecList *V = nullptr, int nv = 0, double *part = nullptr,
                           int ldp = 0, bool hat = false);
int matvec2d_blocks(int nx, int ny, int ell, bool dots);
int matvec2d_dot_walk();
// Right-hand side of every scheme on the unit square (the first rows, zeros after).
hipError_t launch_build_rhs2d(double *b, const double *u0, const double *v0, int nx, int ny,
                              int ell, Scheme sc, double kappa, double tau, hipStream_t st);


}  // namespace aao
