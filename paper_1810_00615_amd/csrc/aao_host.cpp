// Host runtime and C ABI of libaao (declared in include/aao.h).
//
// The context owns every device buffer: the twiddle table of the time FFT, the
// half spectrum of the preconditioner apply, the GMRES basis (stored
// unnormalised, with per-vector scales kept on the device), the search
// directions Z of flexible GMRES, reduction partials and a few scalars.  Every
// operation is enqueued on the context stream; GMRES synchronises once per
// Arnoldi step to read the new Hessenberg column (j+2 doubles) for the Givens
// update on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/aao.h"
#include "aao_internal.h"
#include "batch.h"

using namespace aao;

namespace {

constexpr int kMaxRestart = 63;
constexpr int kPartStride = 16384;   // partials per value (dot and fused-matvec blocks)
constexpr int kSmallStride = 80;   // doubles per small-scalar array
constexpr int kSmallArrays = 11;
// k_reduce_small reads its partials with one workgroup; from this many values on, one
// workgroup per value sums them first (a single workgroup's bandwidth bounds it there)
constexpr int kPreSumValues = 6;

struct Status {
    aao_status st;
};

}  // namespace

struct aao_ctx_s {
    int64_t n = 0, ell = 0;      // n: unknowns per time level (nx ny on the unit square)
    int nx = 0, ny = 0;          // unit square (aao_create_2d); ny = 0 in one dimension
    double *twy = nullptr;       // twiddles of the sine transform's length 2 (ny + 1)
    bool hat = false;            // unit square: operators in sine coordinates along y
    double *bhat = nullptr;      // GMRES right-hand side in those coordinates
    double tau = 0.0;
    int scheme = 0;
    double kappa = 1.0;
    int prec = AAO_PREC_FP64;
    int neumann = 0;
    Scheme sc{};
    hipStream_t st = nullptr;
    int device = 0;
    bool broken = false;
    std::string err;

    double *tw = nullptr;        // ell complex twiddles
    double *tauk = nullptr;      // variable steps (device, ell) or null
    double *sigk = nullptr;      // tau_k - tau (device, ell)
    void *spec = nullptr;        // half spectrum (the solves' output side)
    void *spec_in = nullptr;     // single-precision input spectrum (AAO_PREC_MIXED_IN)
    int lds = 0;
    int *fail = nullptr;         // shifted-solve breakdown flag
    double *sym = nullptr;       // per-row d_j, e_j of the shifted solves
    double sym_kappa = NAN;      // kappa the table was built for
    void *ptab = nullptr;        // partition tables of the shifted solves
    double ptab_kappa = NAN;     // ... built for this kappa,
    int ptab_cw = -1;            // chunk width
    int ptab_single = -1;        // and arithmetic

    // GMRES workspace
    int m_alloc = 0;
    double *V = nullptr, *Z = nullptr, *W = nullptr;
    double *part = nullptr;      // value-major block partials, ldp per value
    int nblk = 0, ldp = 0;
    double *hbuf = nullptr;      // mapped pinned host buffer (k_reduce_small results)
    double *hdev = nullptr;      // its device view
    double *small = nullptr;     // d | h1 | h2 | c | vs | hcol | y
    double *tmpn = nullptr;      // n-vector scratch
    int *dmodes = nullptr;
    double *damps = nullptr;
    int nmodes_alloc = 0;
    double *segpart = nullptr;   // per-segment partials of the checkpointed gradient
    int nseg_alloc = 0;

    // lengths that are not powers of two: Bluestein transforms (the batched
    // kernels with a batch of one)
    bool bluestein = false;
    double *ntmp = nullptr;      // r - E z of a Neumann term (Bluestein lengths)
    BProb *bl_prob = nullptr;
    int2 *bl_tiles = nullptr;
    int bl_ntiles = 0;
    double *bl_chirp = nullptr, *bl_bhat = nullptr, *bl_tw = nullptr;

    // per-kernel timing (aao_set_timing): event pairs recorded around launches
    unsigned timing = 0;         // bit k: kernel id k is timed
    struct Pending {
        int id;
        double bytes;
        hipEvent_t e0, e1;
    };
    std::vector<hipEvent_t> ev_pool;
    std::vector<Pending> ev_pending;
    double t_total[AAO_NUM_KERNELS] = {};
    long long t_count[AAO_NUM_KERNELS] = {};
    double t_bytes[AAO_NUM_KERNELS] = {};
    double seq = 0.0;   // sequence number of the last k_reduce_small launch

    // launch shapes per precision mode (aao_set_config / aao_tune); -1 = default
    int cfg[4][AAO_NUM_CFG] = {
        {-1, -1, -1, -1}, {-1, -1, -1, -1}, {-1, -1, -1, -1}, {-1, -1, -1, -1}};
    int cf(int kind) const { return cfg[prec][kind]; }

    size_t N() const { return (size_t)n * (size_t)ell; }
    double *sd() { return small; }
    double *sh1() { return small + kSmallStride; }
    double *sh2() { return small + 2 * kSmallStride; }
    double *sc_() { return small + 3 * kSmallStride; }
    double *svs() { return small + 4 * kSmallStride; }
    double *shcol() { return small + 5 * kSmallStride; }
    double *sy() { return small + 6 * kSmallStride; }
    double *sa() { return small + 7 * kSmallStride; }    // re-orthogonalisation coefficients
    double *scv() { return small + 8 * kSmallStride; }   // update-pass coefficients (v_j)
    double *scw() { return small + 9 * kSmallStride; }   // update-pass coefficients (w1)
    double *spsum() { return small + 10 * kSmallStride; }   // pre-summed partials
};

#define AAO_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);               \
            ctx->broken = true;                                                         \
            return AAO_ERR_HIP;                                                         \
        }                                                                               \
    } while (0)

static hipEvent_t ev_get(aao_ctx ctx)
{
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    // timing-only events: no system-scope fence (cache writeback) when recorded
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Launch `call` on the context stream; if kernel `id` is timed, bracket it with
// events and record its algorithmic bytes (each operand read or written once).
#define AAO_LAUNCH_B(id, bytes, call)                                                   \
    do {                                                                                \
        hipEvent_t e0_ = nullptr, e1_ = nullptr;                                        \
        const bool tm_ = (ctx->timing >> (id)) & 1u;                                    \
        if (tm_) {                                                                      \
            e0_ = ev_get(ctx);                                                          \
            e1_ = ev_get(ctx);                                                          \
            if (e0_) (void)hipEventRecord(e0_, ctx->st);                                \
        }                                                                               \
        AAO_HIP(call);                                                                  \
        if (tm_ && e0_ && e1_) {                                                        \
            (void)hipEventRecord(e1_, ctx->st);                                         \
            ctx->ev_pending.push_back({(id), (double)(bytes), e0_, e1_});               \
        }                                                                               \
    } while (0)

#define AAO_TRY(expr)                                                                   \
    do {                                                                                \
        aao_status s_ = (expr);                                                         \
        if (s_ < 0) return s_;                                                          \
    } while (0)

static aao_status arg_err(aao_ctx ctx, const char *msg)
{
    if (ctx) ctx->err = msg;
    return AAO_ERR_ARG;
}

static aao_status unsupported_2d(aao_ctx ctx)
{
    ctx->err = "not available on a unit-square context";
    return AAO_ERR_UNSUPPORTED;
}

static bool overlap(const void *a, const void *b, size_t bytes)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + bytes && pb < pa + bytes;
}

static aao_status dev_alloc(aao_ctx ctx, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        ctx->err = std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e);
        return AAO_ERR_ALLOC;
    }
    return AAO_OK;
}

namespace aao {
// Block coefficients of a scheme constant (Sec. 2): the Toeplitz blocks
// A_m = a_m M + b_m kappa K, the start-up rows and the block above the diagonal.
//   heat: eq. monolithicheat read as A_0 = M + tau K, A_1 = -M;
//   BD2:  system C_BD2, A_0 = M + tau^2 K, A_1 = -2M, A_2 = M;
//   BD4:  system C_BD4, A_0 = 2M + tau^2 K, A_1 = -5M, A_2 = 4M, A_3 = -M, start-up
//         rows B = M + tau^2 K (first row) and C = -2M, B (second row);
//   CD:   system C_CD, M u_{k-1} + (tau^2 K - 2M) u_k + M u_{k+1}.
bool make_scheme(int scheme, double tau, Scheme *out)
{
    Scheme s{};
    s.id = scheme;
    const double t2 = tau * tau;
    if (scheme == AAO_HEAT_IE) {
        s.s = 1;
        s.a[0] = 1.0;  s.b[0] = tau;
        s.a[1] = -1.0; s.b[1] = 0.0;
    } else if (scheme == AAO_WAVE_BD2) {
        s.s = 2;
        s.a[0] = 1.0;  s.b[0] = t2;
        s.a[1] = -2.0; s.b[1] = 0.0;
        s.a[2] = 1.0;  s.b[2] = 0.0;
    } else if (scheme == AAO_WAVE_BD4) {
        s.s = 3;
        s.a[0] = 2.0;  s.b[0] = t2;
        s.a[1] = -5.0; s.b[1] = 0.0;
        s.a[2] = 4.0;  s.b[2] = 0.0;
        s.a[3] = -1.0; s.b[3] = 0.0;
        s.nst = 2;
        s.sa[0][0] = 1.0;  s.sb[0][0] = t2;           // B
        s.sa[1][0] = 1.0;  s.sb[1][0] = t2;           // B
        s.sa[1][1] = -2.0;                             // C
    } else if (scheme == AAO_WAVE_CD) {
        s.s = 1;
        s.a[0] = -2.0; s.b[0] = t2;
        s.a[1] = 1.0;  s.b[1] = 0.0;
        s.up = 1;
        s.au = 1.0;    s.bu = 0.0;
    } else {
        return false;
    }
    *out = s;
    return true;
}
}  // namespace aao

static void scheme_of(aao_ctx ctx) { make_scheme(ctx->scheme, ctx->tau, &ctx->sc); }

static void free_workspace(aao_ctx ctx)
{
    (void)hipFree(ctx->V);
    (void)hipFree(ctx->Z);
    (void)hipFree(ctx->W);
    ctx->V = ctx->Z = ctx->W = nullptr;
    ctx->m_alloc = 0;
}

static aao_status ensure_workspace(aao_ctx ctx, int m)
{
    if (ctx->m_alloc >= m) return AAO_OK;
    free_workspace(ctx);
    const size_t N = ctx->N();
    AAO_TRY(dev_alloc(ctx, (void **)&ctx->V, sizeof(double) * N * (m + 1)));
    AAO_TRY(dev_alloc(ctx, (void **)&ctx->Z, sizeof(double) * N * m));
    AAO_TRY(dev_alloc(ctx, (void **)&ctx->W, sizeof(double) * N));
    ctx->m_alloc = m;
    return AAO_OK;
}

// ---------------------------------------------------------------- reductions

// sum over all elements of a.b -> host
static aao_status dot_host(aao_ctx ctx, const double *a, const double *b, double *out)
{
    const size_t N = ctx->N();
    const int nb = dot_blocks(N);
    AAO_HIP(launch_dot1_parts(a, b, N, ctx->part, ctx->st));
    AAO_HIP(launch_reduce_parts(ctx->part, nb, 1, 1, ctx->sd(), ctx->st));
    AAO_HIP(hipMemcpyAsync(out, ctx->sd(), sizeof(double), hipMemcpyDeviceToHost, ctx->st));
    AAO_HIP(hipStreamSynchronize(ctx->st));
    return AAO_OK;
}

// algorithmic bytes: one ell x n FP64 vector, and the half spectrum at the current
// storage precision
static double vec_bytes(aao_ctx ctx) { return 8.0 * (double)ctx->N(); }
// Element types of the preconditioner apply per precision mode: the forward transform
// and the spectrum it writes (input side), the solves' output spectrum and the inverse
// transform (output side), the solve arithmetic.
static bool in_single(int prec) { return prec != AAO_PREC_FP64; }
static bool out_single(int prec) { return prec == AAO_PREC_MIXED || prec == AAO_PREC_FP32; }
static bool arith_single(int prec) { return prec == AAO_PREC_FP32; }
static double spec_bytes(aao_ctx ctx, bool single)
{
    return (single ? 8.0 : 16.0) * (double)(ctx->ell / 2 + 1) * (double)ctx->n;
}
static double spec_in_bytes(aao_ctx ctx) { return spec_bytes(ctx, in_single(ctx->prec)); }
static double spec_out_bytes(aao_ctx ctx) { return spec_bytes(ctx, out_single(ctx->prec)); }
// the spectrum the forward transform writes: a separate single-precision buffer when
// only the input side is single precision, else the solves work in place
static void *in_spec(aao_ctx ctx)
{
    return in_single(ctx->prec) && !out_single(ctx->prec) ? ctx->spec_in : ctx->spec;
}

// --------------------------------------------------------------- operators

static aao_status apply_A_impl(aao_ctx ctx, const double *x, double *y, const double *bsub,
                               int transpose)
{
    if (ctx->ny > 0) {
        AAO_LAUNCH_B(AAO_K_MATVEC, vec_bytes(ctx) * (bsub ? 3 : 2),
                     launch_matvec2d(x, y, bsub, ctx->nx, ctx->ny, (int)ctx->ell, ctx->sc,
                                     ctx->kappa, transpose, ctx->st, nullptr, 0, nullptr, 0,
                                     ctx->hat));
        return AAO_OK;
    }
    AAO_LAUNCH_B(AAO_K_MATVEC, vec_bytes(ctx) * (bsub ? 3 : 2),
                 launch_matvec(x, y, bsub, (int)ctx->n, (int)ctx->ell, ctx->sc,
                                           ctx->kappa, ctx->tauk, transpose, ctx->st,
                                           ctx->cf(AAO_CFG_MATVEC)));
    return AAO_OK;
}

static BatchLaunch bl_launch(aao_ctx ctx)
{
    BatchLaunch L{};
    L.probs = ctx->bl_prob;
    L.count = 1;
    L.ftiles = ctx->bl_tiles;
    L.nftiles = ctx->bl_ntiles;
    L.chirp = ctx->bl_chirp;
    L.bhat = ctx->bl_bhat;
    L.tw = ctx->bl_tw;
    return L;
}

// Rows of the shifted solves: n unknowns, one row per frequency in one dimension; on
// the unit square nx unknowns and ny rows (sine modes in y) per frequency, row q of
// frequency j at spectrum offset j lds + q nx.
static int solve_n(aao_ctx ctx) { return ctx->ny > 0 ? ctx->nx : (int)ctx->n; }
static int solve_rpf(aao_ctx ctx) { return ctx->ny > 0 ? ctx->ny : 1; }
static int solve_sub(aao_ctx ctx) { return ctx->ny > 0 ? ctx->nx : 0; }

// rebuild the per-row symbol table after a change of kappa; the stream is
// synchronised so that later work on any stream sees the table
static aao_status refresh_symbols(aao_ctx ctx)
{
    if (ctx->sym_kappa == ctx->kappa) return AAO_OK;
    AAO_HIP(launch_symbols(ctx->sym, solve_n(ctx), (int)ctx->ell, ctx->sc, ctx->kappa, ctx->st,
                           ctx->ny));
    AAO_HIP(hipStreamSynchronize(ctx->st));
    ctx->sym_kappa = ctx->kappa;
    return AAO_OK;
}

// rebuild the partition tables of the shifted solves for launch shape `cfg` after a
// change of kappa, chunk width or arithmetic (synchronised like the symbols)
static aao_status refresh_tables(aao_ctx ctx, int cfg, bool sync)
{
    const int n = solve_n(ctx);
    cfg = solve_effective_config(cfg, n);
    int cw = 0, nt = 0, stg = 0;
    solve_config_shape(cfg, &cw, &nt, &stg);
    const int single = arith_single(ctx->prec) ? 1 : 0;
    if (ctx->ptab_kappa == ctx->kappa && ctx->ptab_cw == cw && ctx->ptab_single == single)
        return AAO_OK;
    AAO_TRY(refresh_symbols(ctx));
    AAO_HIP(launch_solve_tables(ctx->sym, n, (int)ctx->ell, cfg, single != 0, ctx->ptab, ctx->st,
                                solve_rpf(ctx)));
    if (sync) AAO_HIP(hipStreamSynchronize(ctx->st));
    ctx->ptab_kappa = ctx->kappa;
    ctx->ptab_cw = cw;
    ctx->ptab_single = single;
    return AAO_OK;
}

static aao_status launch_small(aao_ctx ctx, int mode, int nv, int nblk);

// z = C^{-1} (s r - E zprev)  (one circulant apply; s from in_scale).  With
// first_norm (power-of-two ell, no zprev, in_scale unused): the forward transform
// also forms ||r||^2, the fused reduction sets s = 1/||r|| on the device (mode 4 of
// k_reduce_small) and the inverse transform applies s to its output -- the first
// basis vector of a zero-initial-guess solve, whose norm costs no separate pass.
static aao_status pinv_once(aao_ctx ctx, const double *r, const double *in_scale,
                            const double *zprev, double *z, int transpose, bool first_norm = false)
{
    const bool sin = in_single(ctx->prec), sout = out_single(ctx->prec);
    const bool sar = arith_single(ctx->prec);
    const int n = (int)ctx->n, ell = (int)ctx->ell;
    const int sn = solve_n(ctx), rpf = solve_rpf(ctx), sub = solve_sub(ctx);
    void *ispec = in_spec(ctx);
    // single-precision input side: the forward transform's spectrum lives in z, which
    // nothing reads before the inverse transform overwrites it, so the apply touches no
    // more memory than the FP64 one (the 64 MB of cache it would otherwise displace
    // slow the transforms down by a fifth)
    if (ispec == ctx->spec_in && !zprev && !ctx->bluestein && (ctx->ny == 0 || ctx->hat) &&
        (double)(ctx->ell / 2 + 1) * ctx->lds <= (double)ctx->N())
        ispec = z;
    AAO_TRY(refresh_symbols(ctx));
    AAO_TRY(refresh_tables(ctx, ctx->cf(AAO_CFG_SHIFTED_SOLVE), true));
    const double solve_bytes = spec_in_bytes(ctx) + spec_out_bytes(ctx);
    // unit square: C^{-1} = S_y F^{-1} [solves] F S_y (S_y the sine transform in y,
    // which commutes with the time transform F); in sine coordinates (GMRES) the
    // middle factor alone
    if (ctx->ny > 0 && zprev) return AAO_ERR_UNSUPPORTED;
    const bool sq = ctx->ny > 0 && !ctx->hat;
    if (sq) {
        // (S_y r goes to z, which the time transform reads before the inverse transform
        // overwrites it: no extra vector in the working set)
        AAO_LAUNCH_B(AAO_K_SINE_Y, 2 * vec_bytes(ctx),
                     launch_dst_y(r, z, ctx->nx, ctx->ny, ell, ctx->twy, ctx->st));
        r = z;
    }
    if (ctx->bluestein) {
        const BatchLaunch L = bl_launch(ctx);
        if (zprev) {
            // a Neumann term: the Bluestein tiles transform r - E z_prev, formed first
            if (!ctx->ntmp) AAO_TRY(dev_alloc(ctx, (void **)&ctx->ntmp, sizeof(double) * ctx->N()));
            AAO_HIP(launch_neumann_rhs(r, in_scale, zprev, ctx->sigk, ctx->kappa, n, ell,
                                       ctx->ntmp, ctx->st));
            r = ctx->ntmp;
            in_scale = nullptr;
        }
        AAO_LAUNCH_B(AAO_K_FFT_FWD, vec_bytes(ctx) + spec_in_bytes(ctx),
                     batch_fft_fwd(L, r, in_scale, 0, ispec, sin, ctx->st));
        AAO_LAUNCH_B(AAO_K_SHIFTED_SOLVE, solve_bytes,
                   launch_shifted_solve(ispec, ctx->spec, ctx->lds, sin, sout, sar, sn, ell, ctx->sym,
                                        ctx->ptab, transpose, ctx->fail, ctx->st,
                                        ctx->cf(AAO_CFG_SHIFTED_SOLVE), rpf, sub));
        AAO_LAUNCH_B(AAO_K_FFT_INV, vec_bytes(ctx) + spec_out_bytes(ctx),
                     batch_fft_inv(L, ctx->spec, z, sout, ctx->st));
        if (sq)
            AAO_LAUNCH_B(AAO_K_SINE_Y, 2 * vec_bytes(ctx),
                         launch_dst_y(z, z, ctx->nx, ctx->ny, ell, ctx->twy, ctx->st));
        return AAO_OK;
    }
    AAO_LAUNCH_B(AAO_K_FFT_FWD, vec_bytes(ctx) * (zprev ? 2 : 1) + spec_in_bytes(ctx),
               launch_fft_fwd(r, first_norm ? nullptr : in_scale, zprev, ctx->sigk, ctx->kappa,
                              n, ell, ispec, ctx->lds, sin, ctx->tw, ctx->st,
                              ctx->cf(AAO_CFG_FFT_FWD), first_norm ? ctx->part : nullptr));
    if (first_norm)
        AAO_TRY(launch_small(ctx, 4, 1, fft_fwd_blocks(ell, n, sin, ctx->cf(AAO_CFG_FFT_FWD))));
    AAO_LAUNCH_B(AAO_K_SHIFTED_SOLVE, solve_bytes,
               launch_shifted_solve(ispec, ctx->spec, ctx->lds, sin, sout, sar, sn, ell, ctx->sym,
                                    ctx->ptab, transpose, ctx->fail, ctx->st,
                                    ctx->cf(AAO_CFG_SHIFTED_SOLVE), rpf, sub));
    AAO_LAUNCH_B(AAO_K_FFT_INV, vec_bytes(ctx) + spec_out_bytes(ctx),
               launch_fft_inv(ctx->spec, ctx->lds, sout, z, n, ell, ctx->tw, ctx->st,
                              ctx->cf(AAO_CFG_FFT_INV), first_norm ? in_scale : nullptr));
    if (sq)
        AAO_LAUNCH_B(AAO_K_SINE_Y, 2 * vec_bytes(ctx),
                     launch_dst_y(z, z, ctx->nx, ctx->ny, ell, ctx->twy, ctx->st));
    return AAO_OK;
}


// ---------------------------------------------------------------- autotuner

namespace {

using TuneKey = std::tuple<int, int, int, int64_t, int64_t>;   // device, kind, prec, n, ell

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
bool g_tune_file_read = false;
std::string g_tune_path;   // aao_set_tune_cache; empty: per-process cache only

const char *tune_file() { return g_tune_path.empty() ? nullptr : g_tune_path.c_str(); }

// caller holds g_tune_mu
void tune_read_file(int device)
{
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char *path = tune_file();
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    int kind, prec, code;
    long long n, ell;
    double us;
    while (std::fscanf(f, "%d %d %lld %lld %d %lf", &kind, &prec, &n, &ell, &code, &us) == 6)
        g_tune[TuneKey(device, kind, prec, n, ell)] = code;
    std::fclose(f);
}

void tune_append_file(int kind, int prec, int64_t n, int64_t ell, int code, double us)
{
    const char *path = tune_file();
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %lld %lld %d %.3f\n", kind, prec, (long long)n, (long long)ell, code, us);
    std::fclose(f);
}

// size key of the tuning cache: n, or -(ny 2^20 + nx) on the unit square
int64_t tune_n(aao_ctx ctx)
{
    return ctx->ny > 0 ? -(((int64_t)ctx->ny << 20) + ctx->nx) : ctx->n;
}

// admissible codes of one kernel for the context's sizes and precision mode
std::vector<int> tune_candidates(aao_ctx ctx, int kind)
{
    std::vector<int> out;
    const bool single = kind == AAO_CFG_FFT_INV ? out_single(ctx->prec) : in_single(ctx->prec);
    if (kind == AAO_CFG_SHIFTED_SOLVE) {
        for (int c = 0; c < solve_num_configs(); ++c)
            if (solve_config_ok(c, solve_n(ctx))) out.push_back(c);
    } else if (kind == AAO_CFG_MATVEC) {
        // the generic and the unit-square matvecs have one launch shape
        if (!scheme_generic(ctx->sc) && ctx->ny == 0)
            for (int c = 0; c < matvec_num_configs(); ++c) out.push_back(c);
    } else if (!ctx->bluestein) {
        int buf[32];
        const int k = fft_configs((int)ctx->ell, (int)ctx->n, single, buf, 32);
        for (int i = 0; i < k && i < 32; ++i) out.push_back(buf[i]);
    }
    return out;
}

bool config_valid(aao_ctx ctx, int kind, int code)
{
    if (code == -1) return true;
    for (int c : tune_candidates(ctx, kind))
        if (c == code) return true;
    return false;
}

}  // namespace

namespace aao {
bool tune_cache_get(int device, int kind, int prec, int64_t n, int64_t ell, int *code)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_read_file(device);
    auto it = g_tune.find(TuneKey(device, kind, prec, n, ell));
    if (it == g_tune.end()) return false;
    *code = it->second;
    return true;
}

void tune_cache_put(int device, int kind, int prec, int64_t n, int64_t ell, int code, double us)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[TuneKey(device, kind, prec, n, ell)] = code;
    tune_append_file(kind, prec, n, ell, code, us);
}
}  // namespace aao

static aao_status launch_kind(aao_ctx ctx, int kind, int code, double *buf)
{
    if (kind == AAO_CFG_MATVEC) {
        AAO_HIP(launch_matvec(buf, buf + ctx->N(), nullptr, (int)ctx->n, (int)ctx->ell, ctx->sc,
                              ctx->kappa, ctx->tauk, 0, ctx->st, code));
        return AAO_OK;
    }
    const bool sin = in_single(ctx->prec), sout = out_single(ctx->prec);
    const bool sar = arith_single(ctx->prec);
    const int n = (int)ctx->n, ell = (int)ctx->ell;
    if (kind == AAO_CFG_FFT_FWD)
        AAO_HIP(launch_fft_fwd(buf, nullptr, nullptr, ctx->sigk, ctx->kappa, n, ell, in_spec(ctx),
                               ctx->lds, sin, ctx->tw, ctx->st, code));
    else if (kind == AAO_CFG_SHIFTED_SOLVE) {
        AAO_TRY(refresh_tables(ctx, code, false));
        AAO_HIP(launch_shifted_solve(in_spec(ctx), ctx->spec, ctx->lds, sin, sout, sar,
                                     solve_n(ctx), ell, ctx->sym, ctx->ptab, 0, nullptr, ctx->st,
                                     code, solve_rpf(ctx), solve_sub(ctx)));
    }
    else
        AAO_HIP(launch_fft_inv(ctx->spec, ctx->lds, sout, buf, n, ell, ctx->tw, ctx->st, code));
    return AAO_OK;
}

static aao_status tune_impl(aao_ctx ctx, int reps, double *buf)
{
    AAO_TRY(refresh_symbols(ctx));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    AAO_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return arg_err(ctx, "hipEventCreate failed");
    }
    aao_status s = AAO_OK;
    for (int kind = 0; kind < AAO_NUM_CFG && s == AAO_OK; ++kind) {
        const TuneKey key(ctx->device, kind, ctx->prec, tune_n(ctx), ctx->ell);
        {
            std::lock_guard<std::mutex> g(g_tune_mu);
            tune_read_file(ctx->device);
            auto it = g_tune.find(key);
            if (it != g_tune.end() && config_valid(ctx, kind, it->second)) {
                ctx->cfg[ctx->prec][kind] = it->second;
                continue;
            }
        }
        const std::vector<int> cand = tune_candidates(ctx, kind);
        if (cand.empty()) continue;
        int best = -1;
        double best_ms = 0.0;
        for (int code : cand) {
            if ((s = launch_kind(ctx, kind, code, buf)) != AAO_OK) break;   // warm-up
            if (hipEventRecord(e0, ctx->st) != hipSuccess) { s = AAO_ERR_HIP; break; }
            for (int r = 0; r < reps && s == AAO_OK; ++r) s = launch_kind(ctx, kind, code, buf);
            if (s != AAO_OK) break;
            float ms = 0.0f;
            if (hipEventRecord(e1, ctx->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                s = AAO_ERR_HIP;
                break;
            }
            if (best < 0 || ms < best_ms) {
                best = code;
                best_ms = ms;
            }
        }
        if (s != AAO_OK) break;
        ctx->cfg[ctx->prec][kind] = best;
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[key] = best;
        tune_append_file(kind, ctx->prec, tune_n(ctx), ctx->ell, best, 1e3 * best_ms / reps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s == AAO_ERR_HIP) {
        ctx->broken = true;
        if (ctx->err.empty()) ctx->err = "HIP error while tuning";
    }
    return s;
}

// Neumann recurrence of eq. preconapprox1: z_0 = C^{-1} r, z_m = C^{-1}(r - E z_{m-1}).
// The forward transform reads z_{m-1} completely before the inverse transform
// overwrites it, so the recurrence runs in place.
static aao_status pinv_impl(aao_ctx ctx, const double *r, const double *in_scale, double *z,
                            int order, int transpose, bool first_norm = false)
{
    AAO_TRY(pinv_once(ctx, r, in_scale, nullptr, z, transpose, first_norm));
    if (ctx->tauk)
        for (int m = 0; m < order; ++m) AAO_TRY(pinv_once(ctx, r, in_scale, z, z, transpose));
    return AAO_OK;
}

// fused fixed-order reduction of ctx->part + Krylov scalar update (k_reduce_small)
static aao_status launch_small(aao_ctx ctx, int mode, int nv, int nblk)
{
    ctx->seq += 1.0;
    const SmallArgs sa{mode,       nv,        ctx->sh1(), ctx->sh2(), ctx->sc_(),
                       ctx->svs(), ctx->hdev, ctx->fail,  ctx->sa(),  ctx->scv(),
                       ctx->scw(), ctx->seq};
    const int cnt = mode <= 1 ? nv : (mode >= 5 ? nv + 1 : 1);   // values k_reduce_small sums
    if (cnt >= kPreSumValues && nblk > 1) {
        AAO_HIP(launch_reduce_parts(ctx->part, nblk, ctx->ldp, cnt, ctx->spsum(), ctx->st));
        AAO_HIP(launch_reduce_small(ctx->spsum(), 1, 1, sa, ctx->st));
        return AAO_OK;
    }
    AAO_HIP(launch_reduce_small(ctx->part, nblk, ctx->ldp, sa, ctx->st));
    return AAO_OK;
}

// Wait until the last launch_small's results are in the host buffer: poll its
// sequence number (it is written after every other result, behind a system-scope
// fence) for up to about a millisecond, then fall back to synchronising the stream
// (long steps, and the path that reports launch failures).
static aao_status wait_small(aao_ctx ctx)
{
    volatile double *hb = ctx->hbuf;
    const auto t0 = std::chrono::steady_clock::now();
    while (hb[kHostSeq] != ctx->seq) {
        if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(1000)) {
            AAO_HIP(hipStreamSynchronize(ctx->st));
            break;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return AAO_OK;
}

// ------------------------------------------------------------------ GMRES

static aao_status gmres_core(aao_ctx ctx, const double *b, double *x, int m, double tol,
                             int maxit, aao_info *info, int transpose, bool zero_guess,
                             bool classic, bool early_always);

// On the unit square GMRES runs in sine coordinates along y: S_y is orthonormal and
// its own inverse, so FGMRES on (S_y A S_y) (S_y x) = S_y b takes the same steps with
// the same residual norms, while its operators lose both sine transforms of every
// preconditioner apply (C^{-1} becomes F^{-1} [solves] F) and the 9-point stencils
// become 3-point ones per sine mode.  b is transformed once into a vector of the
// context, x on entry (unless it is a zero guess) and on exit.
static aao_status gmres_impl(aao_ctx ctx, const double *b, double *x, int m, double tol,
                             int maxit, aao_info *info, int transpose, bool zero_guess,
                             bool classic = false, bool early_always = false)
{
    if (ctx->ny == 0 || ctx->hat)
        return gmres_core(ctx, b, x, m, tol, maxit, info, transpose, zero_guess, classic,
                          early_always);
    if (m < 1 || m > kMaxRestart) return arg_err(ctx, "restart must be in [1, 63]");
    if (!(tol >= 0.0) || maxit < 0) return arg_err(ctx, "bad tol / maxit");
    if (!b || !x) return arg_err(ctx, "null vector");
    const size_t N = ctx->N();
    if (overlap(b, x, N * sizeof(double))) return arg_err(ctx, "b and x overlap");
    if (!ctx->bhat) AAO_TRY(dev_alloc(ctx, (void **)&ctx->bhat, sizeof(double) * N));
    const int ell = (int)ctx->ell;
    AAO_LAUNCH_B(AAO_K_SINE_Y, 2 * vec_bytes(ctx),
                 launch_dst_y(b, ctx->bhat, ctx->nx, ctx->ny, ell, ctx->twy, ctx->st));
    if (!zero_guess)
        AAO_LAUNCH_B(AAO_K_SINE_Y, 2 * vec_bytes(ctx),
                     launch_dst_y(x, x, ctx->nx, ctx->ny, ell, ctx->twy, ctx->st));
    ctx->hat = true;
    const aao_status s = gmres_core(ctx, ctx->bhat, x, m, tol, maxit, info, transpose, zero_guess,
                                    classic, early_always);
    ctx->hat = false;
    // back to nodal values, also after a failed solve (x then holds the last iterate)
    AAO_LAUNCH_B(AAO_K_SINE_Y, 2 * vec_bytes(ctx),
                 launch_dst_y(x, x, ctx->nx, ctx->ny, ell, ctx->twy, ctx->st));
    return s;
}

static aao_status gmres_core(aao_ctx ctx, const double *b, double *x, int m, double tol,
                             int maxit, aao_info *info, int transpose, bool zero_guess,
                             bool classic, bool early_always)
{
    if (m < 1 || m > kMaxRestart) return arg_err(ctx, "restart must be in [1, 63]");
    if (!(tol >= 0.0) || maxit < 0) return arg_err(ctx, "bad tol / maxit");
    if (!b || !x) return arg_err(ctx, "null vector");
    const size_t N = ctx->N();
    if (overlap(b, x, N * sizeof(double))) return arg_err(ctx, "b and x overlap");
    AAO_TRY(ensure_workspace(ctx, m));
    hipStream_t st = ctx->st;
    const int n = (int)ctx->n, ell = (int)ctx->ell;
    const int nb = dot_blocks(N), ldp = ctx->ldp;
    volatile double *hb = ctx->hbuf;
    AAO_HIP(hipMemsetAsync(ctx->fail, 0, sizeof(int), st));
    auto small = [&](int mode, int nv, int nblk) { return launch_small(ctx, mode, nv, nblk); };

    // basis V_j (V_0 = b for a zero initial guess) and search directions Z_j
    VecList Vl{}, Zl{};
    for (int j = 0; j <= m; ++j) Vl.p[j] = ctx->V + N * j;
    for (int j = 0; j < m; ++j) Zl.p[j] = ctx->Z + N * j;
    double *V0 = ctx->V;
    const int mcfg = ctx->cf(AAO_CFG_MATVEC);
    // the Toeplitz matvec also forms the first Gram-Schmidt dots and residual norms;
    // the start-up-row and two-sided schemes take a plain matvec and separate passes
    // (on the unit square the Q1 matvec forms them for every scheme)
    const bool sq = ctx->ny > 0;
    const int mvb = sq ? matvec2d_blocks(ctx->nx, ctx->ny, ell, true) : matvec_blocks(n, ell, mcfg);
    const bool fused = mvb <= ldp && (sq || !scheme_generic(ctx->sc));
    // a matvec that also forms the partials of L_q . y (q < cnt; see launch_matvec)
    auto mv_dots = [&](const double *xin, double *out, const double *bs, const VecList *L,
                       int cnt) -> hipError_t {
        return sq ? launch_matvec2d(xin, out, bs, ctx->nx, ctx->ny, ell, ctx->sc, ctx->kappa,
                                    transpose, st, L, cnt, ctx->part, ldp, ctx->hat)
                  : launch_matvec(xin, out, bs, n, ell, ctx->sc, ctx->kappa, ctx->tauk,
                                  transpose, st, mcfg, L, cnt, ctx->part, ldp);
    };
    auto residual = [&](bool store) -> aao_status {
        // V_0 = b - A x, vs_0 = 1/||V_0|| (the norm formed by the same launch); with
        // store false only the norm (the check after a cycle, before a restart is
        // known to be needed)
        if (fused) {
            // a one-entry list equal to the output selects the self-norm (|b - A x|^2)
            double *out = store ? V0 : nullptr;
            VecList self{};
            self.p[0] = out;
            AAO_LAUNCH_B(AAO_K_MATVEC, vec_bytes(ctx) * (store ? 3 : 2),
                         mv_dots(x, out, b, &self, 1));
            return small(3, 0, mvb);
        }
        AAO_TRY(apply_A_impl(ctx, x, V0, b, transpose));
        AAO_HIP(launch_dot1_parts(V0, V0, N, ctx->part, st));
        return small(3, 0, nb);
    };

    // ||b|| and the first residual.  With a zero initial guess on a power-of-two
    // length the norm of b is formed inside the first preconditioner apply
    // (pinv_once, first_norm) and read with the first Hessenberg column; otherwise
    // one synchronisation here.
    aao_info inf{};
    const bool defer_b = zero_guess && !ctx->bluestein && fft_supported_fast(ell) && maxit > 0 &&
                         fft_fwd_blocks(ell, n, in_single(ctx->prec), ctx->cf(AAO_CFG_FFT_FWD)) <= ldp;
    double bnorm = 0.0, beta = 0.0;
    if (zero_guess) Vl.p[0] = b;
    auto check_b = [&]() -> aao_status {
        bnorm = std::sqrt(hb[kHostBB]);
        if (!std::isfinite(bnorm)) {
            ctx->err = "non-finite right-hand side";
            return AAO_ERR_NUMERIC;
        }
        return AAO_OK;
    };
    if (!defer_b) {
        AAO_HIP(launch_dot1_parts(b, b, N, ctx->part, st));
        AAO_TRY(small(4, zero_guess ? 1 : 0, nb));
        if (!zero_guess) AAO_TRY(residual(true));
        AAO_HIP(hipStreamSynchronize(st));
        AAO_TRY(check_b());
        beta = hb[kHostBeta];
        if (bnorm == 0.0) {
            AAO_HIP(launch_fill(x, 0.0, N, st));
            AAO_HIP(hipStreamSynchronize(st));
            inf.converged = 1;
            if (info) *info = inf;
            return AAO_OK;
        }
        inf.rel_resid_true = beta / bnorm;
        inf.rel_resid_est = inf.rel_resid_true;
        if (!std::isfinite(beta)) {
            ctx->err = "non-finite residual";
            return AAO_ERR_NUMERIC;
        }
    } else {
        inf.rel_resid_true = inf.rel_resid_est = 1.0;   // x0 = 0: r0 = b
    }
    bool x_zero = zero_guess;   // x not yet written
    auto finish_zero = [&]() -> aao_status {
        if (x_zero) {
            AAO_HIP(launch_fill(x, 0.0, N, st));
            AAO_HIP(hipStreamSynchronize(st));
        }
        return AAO_OK;
    };
    if (!defer_b && (beta / bnorm <= tol || maxit == 0)) {
        AAO_TRY(finish_zero());
        inf.converged = beta / bnorm <= tol;
        if (info) *info = inf;
        return inf.converged ? AAO_OK : AAO_NOT_CONVERGED;
    }

    // Arnoldi: CGS2 with delayed re-orthogonalisation (two passes over the basis per
    // step) unless `classic` (three passes: project, re-project, update).
    // early_always: the early column check at every step after the first (exercises
    // the path where the check fails and the step completes normally)
    const bool delayed = !classic;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hcol(m + 2), y(m),
        hprov(m + 2);
    bool failed = false;
    while (inf.iters < maxit) {
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        // relative residual estimates of the last two steps (the cycle start counts
        // as step -1; x0 = 0 with the deferred norm of b starts from 1)
        double est_prev = bnorm > 0.0 ? beta / bnorm : 1.0, est_prev2 = 1.0;
        int ahead = -1;   // step whose preconditioner apply is already enqueued
        for (int j = 0; j < m; ++j) {
            const double *Vj = Vl.p[j];
            double *Zj = ctx->Z + N * j;
            double *Vn = ctx->V + N * (j + 1);
            const int nv = j + 1;
            // z_j = P^{-1} v_j (unless already enqueued ahead of the previous step's wait);
            // w = A z_j with the first projection V^T w
            const bool first = defer_b && inf.iters == 0;
            if (ahead != j)
                AAO_TRY(pinv_impl(ctx, Vj, ctx->svs() + j, Zj, ctx->neumann, transpose, first));
            // convergence expected at this step (the last two estimates extrapolated
            // geometrically reach tol): the step's column is then checked before the
            // update pass, and w is not stored unless that check fails.  (A looser
            // margin fires at every step of a slowly converging tail, each false
            // expectation costing a second matvec and a host round trip.)
            // (the unit-square matvec reads w back for dots past its first ones)
            const bool expect = delayed && fused && j > 0 &&
                                (early_always || est_prev * (est_prev / est_prev2) <= tol) &&
                                !(sq && nv > matvec2d_dot_walk());
            if (fused) {
                AAO_LAUNCH_B(AAO_K_MATVEC, vec_bytes(ctx) * (expect ? 1 + nv : 2 + nv),
                             mv_dots(Zj, expect ? nullptr : ctx->W, nullptr, &Vl, nv));
            } else {
                AAO_TRY(apply_A_impl(ctx, Zj, ctx->W, nullptr, transpose));
                AAO_LAUNCH_B(AAO_K_CGS_DOT, vec_bytes(ctx) * (nv + 1),
                             launch_multidot(Vl, nv, ctx->W, N, ctx->part, ldp, st));
            }
            bool provisional = false;   // column from the Pythagorean norm, no update pass
            if (delayed) {
                // CGS2 with the re-orthogonalisation of v_j deferred to this step: one
                // pass writes the final v_j and the once-projected w1 (the next pending
                // vector) and forms the dots that re-orthogonalise w1 in the next step
                AAO_TRY(small(5, nv, fused ? mvb : nb));
                // When the estimates so far predict convergence at this step, look
                // first: with |w1|^2 = |w|^2 - |h|^2 the column is known without the
                // update pass, and if its estimate meets tol the update (whose vectors
                // would go unused) is skipped.  The true residual decides convergence.
                if (expect) {
                    AAO_TRY(wait_small(ctx));
                    double hh = 0.0;
                    for (int i = 0; i <= j; ++i) {
                        hprov[i] = hb[i];
                        hh += hprov[i] * hprov[i];
                    }
                    const double b2 = hb[kHostWW] - hh;
                    hprov[nv] = b2 > 0.0 ? std::sqrt(b2) : 0.0;
                    std::vector<double> tcol(hprov.begin(), hprov.begin() + nv + 1);
                    for (int i = 0; i < j; ++i) {
                        const double t = cs[i] * tcol[i] + sn[i] * tcol[i + 1];
                        tcol[i + 1] = -sn[i] * tcol[i] + cs[i] * tcol[i + 1];
                        tcol[i] = t;
                    }
                    const double den = std::hypot(tcol[j], tcol[j + 1]);
                    const double est = den > 0.0 ? std::fabs(g[j]) * tcol[j + 1] / den / bnorm : 1.0;
                    provisional = std::isfinite(est) && est <= 0.5 * tol;
                }
                if (!provisional) {
                    if (expect)   // w was not stored by the first pass
                        AAO_TRY(apply_A_impl(ctx, Zj, ctx->W, nullptr, transpose));
                    AAO_LAUNCH_B(AAO_K_ARNOLDI_UPDATE, vec_bytes(ctx) * (nv + (j > 0 ? 3 : 2)),
                                 launch_arnoldi_update(Vl, nv, ctx->W, ctx->scv(), ctx->scw(),
                                                       j > 0 ? ctx->V + N * j : nullptr, Vn, N,
                                                       ctx->part, ldp, st));
                    AAO_TRY(small(6, nv, nb));
                    // convergence is not expected at this step: the next step's
                    // preconditioner apply (which needs only the pending vector and its
                    // scale, both on the device) is enqueued before the wait, so the GPU
                    // does not idle through the host's Givens update
                    if (!expect && j + 1 < m && inf.iters + 1 < maxit) {
                        AAO_TRY(pinv_impl(ctx, Vl.p[j + 1], ctx->svs() + j + 1,
                                          ctx->Z + N * (j + 1), ctx->neumann, transpose, false));
                        ahead = j + 1;
                    }
                }
            } else {
                AAO_TRY(small(0, nv, fused ? mvb : nb));
                // CGS2: re-project, form the new (unnormalised) basis vector and its norm
                AAO_LAUNCH_B(AAO_K_CGS_UPDATE_DOT, vec_bytes(ctx) * (nv + 1),
                             launch_update_dot(Vl, nv, ctx->W, ctx->sc_(), N, ctx->part, ldp,
                                               st));
                AAO_TRY(small(1, nv, nb));
                AAO_LAUNCH_B(AAO_K_CGS_UPDATE_NORM, vec_bytes(ctx) * (nv + 2),
                             launch_update_norm(Vl, nv, ctx->W, ctx->sc_(), Vn, N, ctx->part,
                                                ldp, st));
                AAO_TRY(small(2, nv, nb));
            }
            if (!provisional) AAO_TRY(wait_small(ctx));
            if (first) {
                AAO_TRY(check_b());
                if (bnorm == 0.0) {
                    AAO_HIP(launch_fill(x, 0.0, N, st));
                    AAO_HIP(hipStreamSynchronize(st));
                    inf.rel_resid_true = inf.rel_resid_est = 0.0;
                    inf.converged = 1;
                    if (info) *info = inf;
                    return AAO_OK;
                }
                beta = bnorm;
                g[0] = beta;
            }
            for (int i = 0; i <= nv; ++i) hcol[i] = provisional ? hprov[i] : hb[i];
            if (delayed && !provisional) {
                // A z_j = sum_{i<=j} h_i v_i + beta p_{j+1}, and p_{j+1} = sum a_i v_i +
                // alpha v_{j+1} with |p_{j+1}| = 1: the column of the fully
                // re-orthogonalised basis
                const double beta = hcol[nv];
                double aa = 0.0;
                for (int i = 0; i <= j; ++i) {
                    const double ai = hb[kHostA + i];
                    hcol[i] += beta * ai;
                    aa += ai * ai;
                }
                hcol[nv] = beta * std::sqrt(std::max(1.0 - aa, 0.0));
            }
            failed = failed || hb[kHostFail] != 0.0;
            inf.iters++;
            for (int i = 0; i <= nv; ++i)
                if (!std::isfinite(hcol[i])) {
                    ctx->err = "non-finite Hessenberg entry (preconditioner breakdown?)";
                    return AAO_ERR_NUMERIC;
                }
            // Givens update of the least-squares problem
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
                hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
                hcol[i] = t;
            }
            const double den = std::hypot(hcol[j], hcol[j + 1]);
            if (den == 0.0) {
                ctx->err = "GMRES breakdown (zero Hessenberg column)";
                return AAO_ERR_NUMERIC;
            }
            cs[j] = hcol[j] / den;
            sn[j] = hcol[j + 1] / den;
            hcol[j] = den;
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hcol[i];
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            inf.rel_resid_est = std::fabs(g[j + 1]) / bnorm;
            est_prev2 = est_prev;
            est_prev = inf.rel_resid_est;
            if (inf.rel_resid_est <= tol || inf.iters >= maxit) break;
        }
        // x (+)= Z y, y = R^{-1} g
        CoefList yc{};
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * y[l];
            y[i] = s / H[(size_t)i * m + i];
            yc.v[i] = y[i];
        }
        if (x_zero && fused && !sq && matvec_comb_ok(mcfg, k)) {
            // x = Z y formed inside the residual-check launch (x is not read, so no
            // block reads rows another one writes): one pass over Z, b and x
            MatvecComb cb{};
            for (int i = 0; i < k; ++i) {
                cb.z[i] = Zl.p[i];
                cb.c[i] = yc.v[i];
            }
            cb.xout = x;
            AAO_LAUNCH_B(AAO_K_MATVEC, vec_bytes(ctx) * (k + 2),
                         launch_matvec_comb(cb, k, b, n, ell, ctx->sc, ctx->kappa, ctx->tauk,
                                            transpose, st, mcfg, ctx->part, ldp));
            AAO_TRY(small(3, 0, mvb));
        } else {
            AAO_LAUNCH_B(AAO_K_AXPY, vec_bytes(ctx) * (k + (x_zero ? 1 : 2)),
                         launch_multi_axpy(Zl, k, yc, x, N, !x_zero, st));
            AAO_TRY(residual(false));
        }
        x_zero = false;
        Vl.p[0] = V0;
        AAO_TRY(wait_small(ctx));
        beta = hb[kHostBeta];
        failed = failed || hb[kHostFail] != 0.0;
        inf.rel_resid_true = beta / bnorm;
        if (!std::isfinite(beta)) {
            ctx->err = "non-finite residual";
            return AAO_ERR_NUMERIC;
        }
        if (inf.rel_resid_true <= tol) {
            inf.converged = 1;
            break;
        }
        if (inf.iters >= maxit) break;
        AAO_TRY(residual(true));   // the restart vector (same launch, now stored)
        inf.restarts++;
    }
    if (info) *info = inf;
    if (failed) {
        ctx->err = "shifted solve produced non-finite values";
        return AAO_ERR_NUMERIC;
    }
    return inf.converged ? AAO_OK : AAO_NOT_CONVERGED;
}

// A context with n unknowns a level; on the unit square (ny > 0) n = nx ny and the
// shifted solves have ny rows of nx unknowns per frequency.  Arguments are checked by
// the callers.
static aao_status create_impl(int64_t n, int64_t ell, double tau, int scheme, int nx, int ny,
                              aao_ctx *out)
{
    aao_ctx ctx = nullptr;
    try {
        ctx = new aao_ctx_s();
    } catch (...) {
        return AAO_ERR_ALLOC;
    }
    ctx->n = n;
    ctx->nx = nx;
    ctx->ny = ny;
    ctx->ell = ell;
    ctx->tau = tau;
    ctx->scheme = scheme;
    scheme_of(ctx);
    aao_status s = AAO_OK;
    do {
        if (hipGetDevice(&ctx->device) != hipSuccess) {
            s = AAO_ERR_HIP;
            break;
        }
        ctx->lds = (int)((n + 15) / 16 * 16);
        const size_t H = (size_t)ell / 2 + 1;
        if ((s = dev_alloc(ctx, (void **)&ctx->tw, sizeof(double) * 2 * ell)) != AAO_OK) break;
        if ((s = dev_alloc(ctx, &ctx->spec, H * ctx->lds * 2 * sizeof(double))) != AAO_OK) break;
        if ((s = dev_alloc(ctx, (void **)&ctx->fail, sizeof(int))) != AAO_OK) break;
        const int rpf = solve_rpf(ctx);
        if ((s = dev_alloc(ctx, (void **)&ctx->sym, sizeof(double) * 8 * H * rpf)) != AAO_OK) break;
        if ((s = dev_alloc(ctx, &ctx->ptab, solve_table_bytes((int)ell, rpf))) != AAO_OK) break;
        if (ny > 0) {
            if ((s = dev_alloc(ctx, (void **)&ctx->twy, sizeof(double) * 4 * (ny + 1))) != AAO_OK)
                break;
            if (launch_twiddles(ctx->twy, 2 * (ny + 1), 2 * (ny + 1), nullptr) != hipSuccess) {
                s = AAO_ERR_HIP;
                break;
            }
        }
        ctx->nblk = dot_blocks(ctx->N());
        ctx->ldp = kPartStride;
        if ((s = dev_alloc(ctx, (void **)&ctx->part,
                           sizeof(double) * (kMaxVecs + 2) * ctx->ldp)) != AAO_OK) break;
        if (hipHostMalloc((void **)&ctx->hbuf, sizeof(double) * kHostSlots, hipHostMallocMapped) !=
                hipSuccess ||
            hipHostGetDevicePointer((void **)&ctx->hdev, ctx->hbuf, 0) != hipSuccess) {
            (void)hipGetLastError();
            s = AAO_ERR_ALLOC;
            break;
        }
        std::memset(ctx->hbuf, 0, sizeof(double) * kHostSlots);
        if ((s = dev_alloc(ctx, (void **)&ctx->small, sizeof(double) * kSmallArrays * kSmallStride)) != AAO_OK)
            break;
        if ((s = dev_alloc(ctx, (void **)&ctx->tmpn, sizeof(double) * n)) != AAO_OK) break;
        if (!fft_supported_fast((int)ell) && ell >= 17 && ell <= 2048 && n <= 16384) {
            // Bluestein transforms through the batched kernels (batch of one)
            BProb q{};
            q.n = (int)n;
            q.ell = (int)ell;
            q.lds = ctx->lds;
            int M = 512;
            while (M < 2 * q.ell - 1) M *= 2;
            q.M = M;
            q.tau = tau;
            q.kappa = 1.0;
            std::vector<int2> tiles;
            const int Wp = bluestein_pairs(M);
            for (int t = 0; t < (q.n + 2 * Wp - 1) / (2 * Wp); ++t) tiles.push_back({0, t});
            ctx->bl_ntiles = (int)tiles.size();
            if ((s = dev_alloc(ctx, (void **)&ctx->bl_prob, sizeof(BProb))) != AAO_OK) break;
            if ((s = dev_alloc(ctx, (void **)&ctx->bl_tiles, sizeof(int2) * tiles.size())) != AAO_OK) break;
            if ((s = dev_alloc(ctx, (void **)&ctx->bl_chirp, sizeof(double) * 2 * ell)) != AAO_OK) break;
            if ((s = dev_alloc(ctx, (void **)&ctx->bl_bhat, sizeof(double) * 4 * M)) != AAO_OK) break;
            if ((s = dev_alloc(ctx, (void **)&ctx->bl_tw, sizeof(double) * 2 * 4096)) != AAO_OK) break;
            if (hipMemcpy(ctx->bl_prob, &q, sizeof(BProb), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(ctx->bl_tiles, tiles.data(), sizeof(int2) * tiles.size(),
                          hipMemcpyHostToDevice) != hipSuccess ||
                batch_prepare() != hipSuccess ||
                launch_twiddles(ctx->bl_tw, 4096, 4096, nullptr) != hipSuccess ||
                batch_setup_tables(ctx->bl_prob, 1, (int)ell, M, ctx->bl_chirp, ctx->bl_bhat,
                                   nullptr) != hipSuccess) {
                s = AAO_ERR_HIP;
                break;
            }
            ctx->bluestein = true;
        }
        if (launch_twiddles(ctx->tw, (int)ell, (int)ell, nullptr) != hipSuccess ||
            hipMemset(ctx->fail, 0, sizeof(int)) != hipSuccess ||
            hipMemset(ctx->small, 0, sizeof(double) * kSmallArrays * kSmallStride) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess) {
            s = AAO_ERR_HIP;
            break;
        }
    } while (0);
    if (s != AAO_OK) {
        aao_destroy(ctx);
        return s;
    }
    *out = ctx;
    return AAO_OK;
}

static bool scheme_known(int scheme)
{
    return scheme == AAO_HEAT_IE || scheme == AAO_WAVE_BD2 || scheme == AAO_WAVE_BD4 ||
           scheme == AAO_WAVE_CD;
}

// ------------------------------------------------------------------- ABI

extern "C" {

aao_status aao_create(int64_t n, int64_t ell, double tau, int scheme, aao_ctx *out)
{
    if (!out) return AAO_ERR_ARG;
    *out = nullptr;
    if (n < 1 || ell < 1 || !(tau > 0.0) || !std::isfinite(tau) || !scheme_known(scheme))
        return AAO_ERR_ARG;
    if (n > 16384 || ell > 65535 || (double)n * (double)ell > 4.0e9) return AAO_ERR_UNSUPPORTED;
    return create_impl(n, ell, tau, scheme, 0, 0, out);
}

aao_status aao_create_2d(int64_t nx, int64_t ny, int64_t ell, double tau, int scheme,
                         aao_ctx *out)
{
    if (!out) return AAO_ERR_ARG;
    *out = nullptr;
    if (nx < 1 || ny < 1 || ell < 1 || !(tau > 0.0) || !std::isfinite(tau) ||
        !scheme_known(scheme))
        return AAO_ERR_ARG;
    if (nx > 16384 || ny > 2047 || !dst_y_supported((int)ny) || ell > 65535 ||
        (double)nx * (double)ny * (double)ell > 2.0e9 || (double)(ell / 2 + 1) * ny > 2.0e9)
        return AAO_ERR_UNSUPPORTED;
    return create_impl(nx * ny, ell, tau, scheme, (int)nx, (int)ny, out);
}

aao_status aao_destroy(aao_ctx ctx)
{
    if (!ctx) return AAO_OK;
    (void)hipStreamSynchronize(ctx->st);
    for (auto &p : ctx->ev_pending) {
        ctx->ev_pool.push_back(p.e0);
        ctx->ev_pool.push_back(p.e1);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    free_workspace(ctx);
    (void)hipFree(ctx->tw);
    (void)hipFree(ctx->tauk);
    (void)hipFree(ctx->sigk);
    (void)hipFree(ctx->spec);
    (void)hipFree(ctx->spec_in);
    (void)hipFree(ctx->fail);
    (void)hipFree(ctx->sym);
    (void)hipFree(ctx->ptab);
    (void)hipFree(ctx->part);
    if (ctx->hbuf) (void)hipHostFree(ctx->hbuf);
    (void)hipFree(ctx->small);
    (void)hipFree(ctx->tmpn);
    (void)hipFree(ctx->dmodes);
    (void)hipFree(ctx->damps);
    (void)hipFree(ctx->segpart);
    (void)hipFree(ctx->ntmp);
    (void)hipFree(ctx->twy);
    (void)hipFree(ctx->bhat);
    (void)hipFree(ctx->bl_prob);
    (void)hipFree(ctx->bl_tiles);
    (void)hipFree(ctx->bl_chirp);
    (void)hipFree(ctx->bl_bhat);
    (void)hipFree(ctx->bl_tw);
    delete ctx;
    return AAO_OK;
}

aao_status aao_set_stream(aao_ctx ctx, void *stream)
{
    if (!ctx) return AAO_ERR_ARG;
    ctx->st = (hipStream_t)stream;
    return AAO_OK;
}

aao_status aao_set_kappa(aao_ctx ctx, double kappa)
{
    if (!ctx) return AAO_ERR_ARG;
    if (!(kappa > 0.0) || !std::isfinite(kappa)) return arg_err(ctx, "kappa must be > 0");
    ctx->kappa = kappa;
    return AAO_OK;
}

aao_status aao_set_steps(aao_ctx ctx, const double *tau_k)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (ctx->ny > 0) return unsupported_2d(ctx);
    if (!tau_k) {
        (void)hipFree(ctx->tauk);
        (void)hipFree(ctx->sigk);
        ctx->tauk = ctx->sigk = nullptr;
        return AAO_OK;
    }
    if (ctx->scheme != AAO_HEAT_IE) {
        ctx->err = "variable steps are defined for the heat scheme only";
        return AAO_ERR_STATE;
    }
    const size_t ell = (size_t)ctx->ell;
    std::vector<double> sig(ell);
    for (size_t k = 0; k < ell; ++k) {
        if (!(tau_k[k] > 0.0) || !std::isfinite(tau_k[k])) return arg_err(ctx, "steps must be > 0");
        sig[k] = tau_k[k] - ctx->tau;
    }
    if (!ctx->tauk) {
        AAO_TRY(dev_alloc(ctx, (void **)&ctx->tauk, sizeof(double) * ell));
        AAO_TRY(dev_alloc(ctx, (void **)&ctx->sigk, sizeof(double) * ell));
    }
    AAO_HIP(hipMemcpy(ctx->tauk, tau_k, sizeof(double) * ell, hipMemcpyHostToDevice));
    AAO_HIP(hipMemcpy(ctx->sigk, sig.data(), sizeof(double) * ell, hipMemcpyHostToDevice));
    return AAO_OK;
}

aao_status aao_set_precision(aao_ctx ctx, int prec)
{
    if (!ctx) return AAO_ERR_ARG;
    if (prec != AAO_PREC_FP64 && prec != AAO_PREC_MIXED && prec != AAO_PREC_FP32 &&
        prec != AAO_PREC_MIXED_IN)
        return arg_err(ctx, "unknown precision");
    if (prec == AAO_PREC_MIXED_IN && !ctx->spec_in) {
        const size_t H = (size_t)ctx->ell / 2 + 1;
        AAO_TRY(dev_alloc(ctx, &ctx->spec_in, H * ctx->lds * 2 * sizeof(float)));
    }
    ctx->prec = prec;
    return AAO_OK;
}

aao_status aao_set_neumann_order(aao_ctx ctx, int q)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->ny > 0 && q != 0) return unsupported_2d(ctx);
    if (q < 0 || q > 64) return arg_err(ctx, "neumann order must be in [0, 64]");
    ctx->neumann = q;
    return AAO_OK;
}

aao_status aao_project_sine(aao_ctx ctx, int J, const int *modes, const double *amps, double *u0)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (ctx->ny > 0) return unsupported_2d(ctx);
    if (J < 0 || (J > 0 && (!modes || !amps)) || !u0) return arg_err(ctx, "bad sine series");
    for (int m = 0; m < J; ++m)
        if (modes[m] < 1) return arg_err(ctx, "modes must be >= 1");
    if (J > ctx->nmodes_alloc) {
        (void)hipFree(ctx->dmodes);
        (void)hipFree(ctx->damps);
        ctx->dmodes = nullptr;
        ctx->damps = nullptr;
        ctx->nmodes_alloc = 0;
        AAO_TRY(dev_alloc(ctx, (void **)&ctx->dmodes, sizeof(int) * J));
        AAO_TRY(dev_alloc(ctx, (void **)&ctx->damps, sizeof(double) * J));
        ctx->nmodes_alloc = J;
    }
    if (J > 0) {
        AAO_HIP(hipMemcpyAsync(ctx->dmodes, modes, sizeof(int) * J, hipMemcpyHostToDevice, ctx->st));
        AAO_HIP(hipMemcpyAsync(ctx->damps, amps, sizeof(double) * J, hipMemcpyHostToDevice, ctx->st));
    }
    AAO_HIP(launch_project_sine(u0, (int)ctx->n, J, ctx->dmodes, ctx->damps, ctx->st));
    AAO_HIP(hipStreamSynchronize(ctx->st));
    return AAO_OK;
}

aao_status aao_build_rhs(aao_ctx ctx, const double *u0, const double *v0, double *b)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (!u0 || !b) return arg_err(ctx, "null vector");
    if (v0 && ctx->scheme == AAO_WAVE_CD)
        return arg_err(ctx, "the central-difference system takes no initial velocity");
    if (ctx->ny > 0) {
        if (ctx->scheme == AAO_WAVE_BD2 && ctx->ell < 2)
            return arg_err(ctx, "the BD2 right-hand side needs ell >= 2");
        if (ctx->scheme == AAO_WAVE_BD4 && ctx->ell < 3)
            return arg_err(ctx, "the BD4 right-hand side needs ell >= 3");
        if (v0 && ctx->scheme == AAO_HEAT_IE)
            return arg_err(ctx, "the heat system takes no initial velocity");
        AAO_HIP(launch_build_rhs2d(b, u0, v0, ctx->nx, ctx->ny, (int)ctx->ell, ctx->sc, ctx->kappa,
                                   ctx->tau, ctx->st));
        return AAO_OK;
    }
    AAO_HIP(launch_build_rhs(b, u0, v0, (int)ctx->n, (int)ctx->ell, ctx->sc, ctx->kappa, ctx->tau,
                             ctx->st));
    return AAO_OK;
}

aao_status aao_apply_A(aao_ctx ctx, const double *x, double *y, int transpose)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (!x || !y) return arg_err(ctx, "null vector");
    if (overlap(x, y, ctx->N() * sizeof(double))) return arg_err(ctx, "x and y overlap");
    return apply_A_impl(ctx, x, y, nullptr, transpose ? 1 : 0);
}

aao_status aao_apply_Pinv(aao_ctx ctx, const double *r, double *z, int neumann_order,
                          int transpose)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (!r || !z) return arg_err(ctx, "null vector");
    if (neumann_order < 0 || neumann_order > 64) return arg_err(ctx, "bad neumann order");
    if (ctx->ny > 0 && neumann_order != 0) return unsupported_2d(ctx);
    if (overlap(r, z, ctx->N() * sizeof(double))) return arg_err(ctx, "r and z overlap");
    return pinv_impl(ctx, r, nullptr, z, neumann_order, transpose ? 1 : 0);
}

aao_status aao_gmres(aao_ctx ctx, const double *b, double *x, int restart, double tol, int maxit,
                     aao_info *info)
{
    return aao_gmres_ex(ctx, b, x, restart, tol, maxit, 0, info);
}

aao_status aao_gmres_ex(aao_ctx ctx, const double *b, double *x, int restart, double tol,
                        int maxit, int flags, aao_info *info)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (flags & ~(AAO_GMRES_ZERO_GUESS | AAO_GMRES_TRANSPOSE | AAO_GMRES_CGS2_CLASSIC |
                  AAO_GMRES_EARLY_CHECK))
        return arg_err(ctx, "bad flags");
    try {
        return gmres_impl(ctx, b, x, restart, tol, maxit, info,
                          (flags & AAO_GMRES_TRANSPOSE) ? 1 : 0, (flags & AAO_GMRES_ZERO_GUESS) != 0,
                          (flags & AAO_GMRES_CGS2_CLASSIC) != 0,
                          (flags & AAO_GMRES_EARLY_CHECK) != 0);
    } catch (const std::bad_alloc &) {
        return AAO_ERR_ALLOC;
    } catch (...) {
        return AAO_ERR_HIP;
    }
}

aao_status aao_adjoint_solve(aao_ctx ctx, const double *g, double *lam, int restart, double tol,
                             int maxit, aao_info *info)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    try {
        return gmres_impl(ctx, g, lam, restart, tol, maxit, info, 1, false);
    } catch (const std::bad_alloc &) {
        return AAO_ERR_ALLOC;
    } catch (...) {
        return AAO_ERR_HIP;
    }
}

aao_status aao_grad(aao_ctx ctx, const double *u0, const double *v0, const double *U,
                    const double *lam, double *g_u0, double *g_v0, double *g_kappa)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (ctx->ny > 0) return unsupported_2d(ctx);
    if (!U || !lam || !g_u0) return arg_err(ctx, "null vector");
    const int n = (int)ctx->n;
    const double tau = ctx->tau, kap = ctx->kappa;
    // BD2 and BD4 share the start-up row b_1 = (M + tau^2 kappa K)(u0 + tau v0)
    const bool wave = ctx->scheme == AAO_WAVE_BD2 || ctx->scheme == AAO_WAVE_BD4;
    const bool bd2 = wave;
    if (wave && g_kappa && !u0) return arg_err(ctx, "u0 needed for the wave kappa gradient");
    hipStream_t st = ctx->st;
    const double *lam1 = lam, *lam2 = ctx->ell > 1 ? lam + n : nullptr;
    const double *lam3 = ctx->ell > 2 ? lam + 2 * (size_t)n : nullptr;
    if (ctx->scheme == AAO_HEAT_IE) {
        AAO_HIP(launch_mk(lam1, 1.0, 0.0, nullptr, 0.0, 0.0, g_u0, n, st));
    } else if (ctx->scheme == AAO_WAVE_CD) {
        AAO_HIP(launch_mk(lam1, -1.0, 0.0, nullptr, 0.0, 0.0, g_u0, n, st));   // b_1 = -M u0
    } else {
        // BD2: A_0 lam_1 - M lam_2; BD4: B lam_1 - M lam_2 + M lam_3
        const bool bd4 = ctx->scheme == AAO_WAVE_BD4;
        AAO_HIP(launch_mk(lam1, 1.0, tau * tau * kap, lam2, lam2 ? -1.0 : 0.0, 0.0, g_u0, n, st,
                          bd4 ? lam3 : nullptr, 1.0, 0.0));
    }
    if (g_v0) {
        if (wave)
            AAO_HIP(launch_mk(lam1, tau, tau * tau * tau * kap, nullptr, 0.0, 0.0, g_v0, n, st));
        else
            AAO_HIP(launch_fill(g_v0, 0.0, (size_t)n, st));
    }
    if (g_kappa) {
        const int nb = dot_blocks(ctx->N());
        AAO_HIP(launch_grad_kappa_parts(U, lam, n, (int)ctx->ell, ctx->sc, ctx->tauk, ctx->part, nb,
                                        st));
        AAO_HIP(launch_reduce_parts(ctx->part, nb, 1, 1, ctx->sd(), st));
        double s = 0.0;
        AAO_HIP(hipMemcpyAsync(&s, ctx->sd(), sizeof(double), hipMemcpyDeviceToHost, st));
        AAO_HIP(hipStreamSynchronize(st));
        double gk = -s;
        if (bd2) {
            // + lam_1 . tau^2 K (u0 + tau v0)
            AAO_HIP(launch_mk(u0, 0.0, tau * tau, v0, 0.0, v0 ? tau * tau * tau : 0.0, ctx->tmpn, n,
                              st));
            const int nbn = dot_blocks((size_t)n);
            AAO_HIP(launch_dot1_parts(ctx->tmpn, lam1, (size_t)n, ctx->part, st));
            AAO_HIP(launch_reduce_parts(ctx->part, nbn, 1, 1, ctx->sd(), st));
            double t = 0.0;
            AAO_HIP(hipMemcpyAsync(&t, ctx->sd(), sizeof(double), hipMemcpyDeviceToHost, st));
            AAO_HIP(hipStreamSynchronize(st));
            gk += t;
        }
        *g_kappa = gk;
    } else {
        AAO_HIP(hipStreamSynchronize(st));
    }
    return AAO_OK;
}

aao_status aao_grad_checkpointed(aao_ctx ctx, const double *u0, const double *Uck, int stride,
                                 const double *lam, double *g_u0, double *g_kappa, double *U_out)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (ctx->ny > 0) return unsupported_2d(ctx);
    if (ctx->scheme != AAO_HEAT_IE) {
        ctx->err = "checkpointed gradients are implemented for the heat scheme";
        return AAO_ERR_UNSUPPORTED;
    }
    if (stride < 1 || !u0 || !lam || !g_u0) return arg_err(ctx, "bad checkpoint arguments");
    if (ctx->ell > stride && !Uck) return arg_err(ctx, "checkpoint rows missing");
    const int n = (int)ctx->n, ell = (int)ctx->ell;
    hipStream_t st = ctx->st;
    AAO_HIP(launch_mk(lam, 1.0, 0.0, nullptr, 0.0, 0.0, g_u0, n, st));
    if (g_kappa || U_out) {
        const int nseg = (ell + stride - 1) / stride;
        if (nseg > ctx->nseg_alloc) {
            (void)hipFree(ctx->segpart);
            ctx->segpart = nullptr;
            ctx->nseg_alloc = 0;
            AAO_TRY(dev_alloc(ctx, (void **)&ctx->segpart, sizeof(double) * nseg));
            ctx->nseg_alloc = nseg;
        }
        AAO_HIP(hipMemsetAsync(ctx->fail, 0, sizeof(int), st));
        AAO_HIP(launch_heat_segments(u0, Uck, stride, lam, n, ell, ctx->tau, ctx->kappa, ctx->tauk,
                                     ctx->segpart, U_out, ctx->fail, st));
        AAO_HIP(launch_reduce_parts(ctx->segpart, nseg, 1, 1, ctx->sd(), st));
        double s = 0.0;
        int failed = 0;
        AAO_HIP(hipMemcpyAsync(&s, ctx->sd(), sizeof(double), hipMemcpyDeviceToHost, st));
        AAO_HIP(hipMemcpyAsync(&failed, ctx->fail, sizeof(int), hipMemcpyDeviceToHost, st));
        AAO_HIP(hipStreamSynchronize(st));
        if (failed) {
            ctx->err = "non-finite value while recomputing the trajectory";
            return AAO_ERR_NUMERIC;
        }
        if (g_kappa) *g_kappa = -s;
    } else {
        AAO_HIP(hipStreamSynchronize(st));
    }
    return AAO_OK;
}

aao_status aao_set_timing_mask(aao_ctx ctx, unsigned mask)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    AAO_HIP(hipStreamSynchronize(ctx->st));
    for (auto &p : ctx->ev_pending) {
        ctx->ev_pool.push_back(p.e0);
        ctx->ev_pool.push_back(p.e1);
    }
    ctx->ev_pending.clear();
    for (int i = 0; i < AAO_NUM_KERNELS; ++i) {
        ctx->t_total[i] = 0.0;
        ctx->t_count[i] = 0;
        ctx->t_bytes[i] = 0.0;
    }
    ctx->timing = mask & ((1u << AAO_NUM_KERNELS) - 1u);
    return AAO_OK;
}

aao_status aao_set_timing(aao_ctx ctx, int enable)
{
    return aao_set_timing_mask(ctx, enable ? ~0u : 0u);
}

aao_status aao_get_timing_ex(aao_ctx ctx, int kernel, double *total_ms, int64_t *count,
                             double *bytes)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (kernel < 0 || kernel >= AAO_NUM_KERNELS || !total_ms || !count)
        return arg_err(ctx, "bad kernel id / output");
    AAO_HIP(hipStreamSynchronize(ctx->st));
    for (auto &p : ctx->ev_pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
            ctx->t_total[p.id] += ms;
            ctx->t_count[p.id] += 1;
            ctx->t_bytes[p.id] += p.bytes;
        }
        ctx->ev_pool.push_back(p.e0);
        ctx->ev_pool.push_back(p.e1);
    }
    ctx->ev_pending.clear();
    *total_ms = ctx->t_total[kernel];
    *count = ctx->t_count[kernel];
    if (bytes) *bytes = ctx->t_bytes[kernel];
    return AAO_OK;
}

aao_status aao_get_timing(aao_ctx ctx, int kernel, double *total_ms, int64_t *count)
{
    return aao_get_timing_ex(ctx, kernel, total_ms, count, nullptr);
}

aao_status aao_tune(aao_ctx ctx, int reps)
{
    if (!ctx) return AAO_ERR_ARG;
    if (ctx->broken) return AAO_ERR_HIP;
    if (reps < 1 || reps > 1000) return arg_err(ctx, "reps must be in [1, 1000]");
    // scratch: two real ell x n arrays (zeros) for the transforms and the matvec; the
    // half spectrum is workspace and is rewritten by every apply
    double *buf = nullptr;
    AAO_TRY(dev_alloc(ctx, (void **)&buf, 2 * sizeof(double) * ctx->N()));
    aao_status s = AAO_OK;
    const size_t H = (size_t)ctx->ell / 2 + 1;
    if (launch_fill(buf, 0.0, 2 * ctx->N(), ctx->st) != hipSuccess ||
        launch_fill((double *)ctx->spec, 0.0, H * ctx->lds * 2, ctx->st) != hipSuccess ||
        (ctx->spec_in &&
         launch_fill((double *)ctx->spec_in, 0.0, H * ctx->lds, ctx->st) != hipSuccess))
        s = AAO_ERR_HIP;
    if (s == AAO_OK) s = tune_impl(ctx, reps, buf);
    (void)hipStreamSynchronize(ctx->st);
    (void)hipFree(buf);
    if (s == AAO_ERR_HIP) {
        ctx->broken = true;
        if (ctx->err.empty()) ctx->err = "HIP error while tuning";
    }
    return s;
}

aao_status aao_set_tune_cache(const char *path)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_path = path ? path : "";
    g_tune_file_read = false;   // read the (new) file at the next aao_tune
    return AAO_OK;
}

aao_status aao_get_config(aao_ctx ctx, int kind, int *code)
{
    if (!ctx || !code) return AAO_ERR_ARG;
    if (kind < 0 || kind >= AAO_NUM_CFG) return arg_err(ctx, "bad config kind");
    *code = ctx->cfg[ctx->prec][kind];
    return AAO_OK;
}

aao_status aao_set_config(aao_ctx ctx, int kind, int code)
{
    if (!ctx) return AAO_ERR_ARG;
    if (kind < 0 || kind >= AAO_NUM_CFG) return arg_err(ctx, "bad config kind");
    if (!config_valid(ctx, kind, code)) return arg_err(ctx, "launch shape does not fit n, ell");
    ctx->cfg[ctx->prec][kind] = code;
    return AAO_OK;
}

aao_status aao_config_shape(aao_ctx ctx, int kind, int code, int shape[3])
{
    if (!ctx || !shape) return AAO_ERR_ARG;
    if (kind < 0 || kind >= AAO_NUM_CFG) return arg_err(ctx, "bad config kind");
    if (code < 0) return arg_err(ctx, "default shapes have no code");
    if (kind == AAO_CFG_SHIFTED_SOLVE) {
        if (code >= solve_num_configs()) return arg_err(ctx, "bad code");
        solve_config_shape(code, &shape[0], &shape[1], &shape[2]);
    } else if (kind == AAO_CFG_MATVEC) {
        if (code >= matvec_num_configs()) return arg_err(ctx, "bad code");
        shape[0] = 4 << (code % 3);
        shape[1] = code / 3;
        shape[2] = 0;
    } else {
        const int L = (int)ctx->ell / 2;
        shape[0] = code >= 16 ? 8 : (L < 16 ? L : 16);
        shape[1] = 1 << (code & 15);
        shape[2] = 0;
    }
    return AAO_OK;
}

const char *aao_status_string(aao_status st)
{
    switch (st) {
    case AAO_OK: return "ok";
    case AAO_NOT_CONVERGED: return "not converged";
    case AAO_ERR_ARG: return "invalid argument";
    case AAO_ERR_ALLOC: return "device allocation failed";
    case AAO_ERR_HIP: return "HIP runtime error";
    case AAO_ERR_NUMERIC: return "numerical breakdown";
    case AAO_ERR_STATE: return "invalid state";
    case AAO_ERR_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

const char *aao_last_error(aao_ctx ctx)
{
    if (!ctx) return "";
    return ctx->err.c_str();
}

}  // extern "C"
