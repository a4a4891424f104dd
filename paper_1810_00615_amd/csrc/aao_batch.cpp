// Host side of the batched form (declared in include/aao.h, aao_batch_*).
//
// A batch vector concatenates the ell_p x n_p arrays of all problems (offsets
// aligned to 64 elements, see aao_batch_offsets).  Every phase of an Arnoldi
// step is one launch over a work table that spans all problems; converged
// problems are masked out on the device.  The launch sequence of Arnoldi step j
// does not depend on the data, so it is captured once into a hipGraph and
// replayed; the host reads one integer (the number of problems still active)
// after each step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/aao.h"
#include "aao_internal.h"

#include "batch.h"

using namespace aao;

namespace {
constexpr int kBMaxRestart = 63;
}

struct aao_batch_s {
    int count = 0, scheme = 0, prec = AAO_PREC_MIXED;
    std::vector<BProb> hp;
    size_t Ntot = 0, Stot = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    bool use_graph = true;
    // launch shapes (aao_batch_set_config / aao_batch_tune): elements per slab of the
    // Gram-Schmidt, update and solution passes; time levels per matvec tile; Arnoldi
    // steps captured per graph (0 = the rest of the restart cycle)
    int slab = kBatchSlabDefault, mrows = kMatvecRowsDefault, span = kGraphSpanDefault;
    // CGS2 with deferred re-orthogonalisation (two passes per Arnoldi step) unless the
    // solve asks for the three-pass form (AAO_GMRES_CGS2_CLASSIC)
    bool delayed = true;
    std::string err;
    bool broken = false;

    BProb *probs = nullptr;
    int2 *ftiles = nullptr, *rows = nullptr, *pslabs = nullptr, *mranges = nullptr;
    int4 *mtiles = nullptr, *slabs = nullptr;
    int nftiles = 0, nrows = 0, nmtiles = 0, nslabs = 0;
    int row_start[5] = {};
    double *chirp = nullptr, *bhat = nullptr, *tw = nullptr;
    void *spec = nullptr;           // half spectra (the solves' output side)
    void *spec_in = nullptr;        // single-precision input spectra (AAO_PREC_MIXED_IN)
    int *fail = nullptr;

    // GMRES workspace and state
    int m_alloc = 0;
    double *V = nullptr, *Z = nullptr, *W = nullptr;
    double **dV = nullptr, **dZ = nullptr;
    // host sources of the pointer-table updates of a zero-guess cycle (members, so
    // that they outlive the asynchronous copies that read them)
    const double *first_b = nullptr, *first_v = nullptr;
    double *part = nullptr;
    int ldp = kBMaxRestart + 2;
    double *sm = nullptr;           // small per-problem arrays
    double *H = nullptr;
    int *iv = nullptr;              // iters | ksteps | nact
    unsigned char *flags = nullptr; // active | done | bad
    BState bs{};
    std::vector<hipGraphExec_t> graphs;   // by first step: steps [j, j + span) of a cycle
    // the captured steps depend on these: a solve with other values recaptures
    int graph_m = 0, graph_maxit = -1, graph_transpose = -1, graph_delayed = -1, graph_span = -1;
    double graph_tol = -1.0;
    double **dB = nullptr;           // one-entry pointer array for norms of the rhs

    BatchLaunch launch(bool masked) const
    {
        BatchLaunch L;
        L.probs = probs;
        L.count = count;
        L.ftiles = ftiles;
        L.nftiles = nftiles;
        L.rows = rows;
        L.nrows = nrows;
        for (int c = 0; c < 5; ++c) L.row_start[c] = row_start[c];
        L.mtiles = mtiles;
        L.nmtiles = nmtiles;
        L.mrows = mrows;
        L.slabs = slabs;
        L.nslabs = nslabs;
        L.pslabs = pslabs;
        L.mranges = mranges;
        L.active = masked ? flags : nullptr;
        L.chirp = chirp;
        L.bhat = bhat;
        L.tw = tw;
        return L;
    }
};

#define BH(call)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            b->err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
            b->broken = true;                                                             \
            return AAO_ERR_HIP;                                                           \
        }                                                                                 \
    } while (0)

#define BT(expr)                                                                          \
    do {                                                                                  \
        aao_status s_ = (expr);                                                           \
        if (s_ < 0) return s_;                                                            \
    } while (0)

static aao_status balloc(aao_batch b, void **p, size_t bytes)
{
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        b->err = "hipMalloc(" + std::to_string(bytes) + ") failed";
        return AAO_ERR_ALLOC;
    }
    return AAO_OK;
}

template <typename T>
static aao_status upload(aao_batch b, T **dst, const std::vector<T> &src)
{
    BT(balloc(b, (void **)dst, sizeof(T) * std::max<size_t>(src.size(), 1)));
    if (!src.empty())
        BH(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return AAO_OK;
}

static void free_ws(aao_batch b)
{
    for (auto g : b->graphs)
        if (g) (void)hipGraphExecDestroy(g);
    b->graphs.clear();
    b->graph_m = 0;
    (void)hipFree(b->V);
    (void)hipFree(b->Z);
    (void)hipFree(b->W);
    (void)hipFree(b->dV);
    (void)hipFree(b->dZ);
    b->V = b->Z = b->W = nullptr;
    b->dV = b->dZ = nullptr;
    b->m_alloc = 0;
}

static aao_status ensure_ws(aao_batch b, int m)
{
    if (b->m_alloc >= m) return AAO_OK;
    free_ws(b);
    const size_t N = b->Ntot;
    BT(balloc(b, (void **)&b->V, sizeof(double) * N * (m + 1)));
    BT(balloc(b, (void **)&b->Z, sizeof(double) * N * m));
    BT(balloc(b, (void **)&b->W, sizeof(double) * N));
    std::vector<double *> hv(m + 1), hz(m);
    for (int i = 0; i <= m; ++i) hv[i] = b->V + N * i;
    for (int i = 0; i < m; ++i) hz[i] = b->Z + N * i;
    BT(upload(b, &b->dV, hv));
    BT(upload(b, &b->dZ, hz));
    b->m_alloc = m;
    return AAO_OK;
}

// Work tables that depend on the launch shapes: matvec tiles (256 columns x mrows time
// levels) with each problem's tile range, element slabs of `slab` elements with each
// problem's slab range, and the block partials both leave (ldp values each).
static aao_status build_work_tables(aao_batch b)
{
    std::vector<int4> mt, sl;
    std::vector<int2> mr, ps;
    for (int p = 0; p < b->count; ++p) {
        const BProb &q = b->hp[p];
        const int mfirst = (int)mt.size();
        for (int by = 0; by < (q.ell + b->mrows - 1) / b->mrows; ++by)
            for (int bx = 0; bx < (q.n + 255) / 256; ++bx) mt.push_back({p, bx, by, 0});
        mr.push_back({mfirst, (int)mt.size()});
        const size_t Np = (size_t)q.n * q.ell;
        const int first = (int)sl.size();
        for (size_t e0 = 0; e0 < Np; e0 += (size_t)b->slab)
            sl.push_back({p, (int)e0, (int)std::min<size_t>((size_t)b->slab, Np - e0), 0});
        ps.push_back({first, (int)sl.size()});
    }
    (void)hipFree(b->mtiles);
    (void)hipFree(b->slabs);
    (void)hipFree(b->pslabs);
    (void)hipFree(b->mranges);
    (void)hipFree(b->part);
    b->mtiles = b->slabs = nullptr;
    b->pslabs = b->mranges = nullptr;
    b->part = nullptr;
    b->nmtiles = (int)mt.size();
    b->nslabs = (int)sl.size();
    BT(upload(b, &b->mtiles, mt));
    BT(upload(b, &b->slabs, sl));
    BT(upload(b, &b->pslabs, ps));
    BT(upload(b, &b->mranges, mr));
    BT(balloc(b, (void **)&b->part, sizeof(double) * b->ldp * std::max(b->nslabs, b->nmtiles)));
    // captured graphs hold the old tables
    for (auto g : b->graphs)
        if (g) (void)hipGraphExecDestroy(g);
    b->graphs.clear();
    b->graph_m = 0;
    return AAO_OK;
}

// ------------------------------------------------------------------ phases

static aao_status b_pinv(aao_batch b, const double *r, const double *scales, int sstride, double *z,
                         bool masked, int transpose)
{
    const bool sin = b->prec != AAO_PREC_FP64;
    const bool sout = b->prec == AAO_PREC_MIXED || b->prec == AAO_PREC_FP32;
    const bool sar = b->prec == AAO_PREC_FP32;
    void *ispec = sin && !sout ? b->spec_in : b->spec;
    const BatchLaunch L = b->launch(masked);
    BH(batch_fft_fwd(L, r, scales, sstride, ispec, sin, b->st));
    BH(batch_solve(L, ispec, b->spec, sin, sout, sar, b->scheme, transpose, b->fail, b->st));
    BH(batch_fft_inv(L, b->spec, z, sout, b->st));
    return AAO_OK;
}

// One Arnoldi step j for every active problem (the sequence that is captured).
// v0 (step 0 only, may be null): the first basis vector's storage when it is not
// the workspace's own (the right-hand side itself, for a zero initial guess).
static aao_status b_step(aao_batch b, int j, int m, double tol, int transpose,
                         const double *v0 = nullptr)
{
    const size_t N = b->Ntot;
    const BatchLaunch L = b->launch(true);
    const int nv = j + 1;
    BState &s = b->bs;
    const double *Vj = (j == 0 && v0) ? v0 : b->V + N * j;
    double *Zj = b->Z + N * j, *Vn = b->V + N * (j + 1);
    BT(b_pinv(b, Vj, s.vs + j, s.sst, Zj, true, transpose));
    if (b->delayed && nv <= 4) {
        // the first Gram-Schmidt pass (dots of w with the basis and the pending
        // vector) formed by the matvec itself
        BH(batch_matvec(L, Zj, b->W, nullptr, b->scheme, transpose, true, b->st, b->dV, nv,
                        b->part, b->ldp));
        BH(batch_reduce(L, b->part, b->ldp, nv, s.dsum, s.sst, true, b->st, L.mranges));
    } else {
        BH(batch_matvec(L, Zj, b->W, nullptr, b->scheme, transpose, true, b->st));
        BH(batch_cgs(0, L, b->dV, nv, b->W, nullptr, 0, nullptr, b->part, b->ldp, true, b->st));
        BH(batch_reduce(L, b->part, b->ldp, nv, s.dsum, s.sst, true, b->st));
    }
    if (b->delayed) {
        // CGS2 with the re-orthogonalisation deferred by one step: the dots above
        // (with the pending V_j), then one pass that writes the final v_j and the
        // once-projected next vector and forms the dots of its re-orthogonalisation
        BH(batch_small(4, b->count, j, m, tol, s, b->st));
        BH(batch_cgs_delayed(L, b->dV, nv, b->W, s, Vn, b->part, b->ldp, b->st));
        BH(batch_reduce(L, b->part, b->ldp, nv + 1, s.dsum, s.sst, true, b->st));
        BH(batch_small(5, b->count, j, m, tol, s, b->st));
        BH(batch_count_active(s.active, b->count, b->iv + 2 * b->count, b->st));
        return AAO_OK;
    }
    BH(batch_small(0, b->count, j, m, tol, s, b->st));
    BH(batch_cgs(1, L, b->dV, nv, b->W, s.coef, s.sst, nullptr, b->part, b->ldp, true, b->st));
    BH(batch_reduce(L, b->part, b->ldp, nv, s.dsum, s.sst, true, b->st));
    BH(batch_small(1, b->count, j, m, tol, s, b->st));
    BH(batch_cgs(2, L, b->dV, nv, b->W, s.coef, s.sst, Vn, b->part, b->ldp, true, b->st));
    BH(batch_reduce(L, b->part, b->ldp, 1, s.dsum, s.sst, true, b->st));
    BH(batch_small(2, b->count, j, m, tol, s, b->st));
    BH(batch_count_active(s.active, b->count, b->iv + 2 * b->count, b->st));
    return AAO_OK;
}

// true if two batch vectors (Ntot doubles each) share memory
static bool b_overlap(const aao_batch b, const void *p, const void *q)
{
    const auto a = reinterpret_cast<uintptr_t>(p), c = reinterpret_cast<uintptr_t>(q);
    const uintptr_t bytes = sizeof(double) * b->Ntot;
    return a < c + bytes && c < a + bytes;
}

// zero: x0 = 0 whatever x holds (x is only written).  The first cycle then takes
// b itself as its first basis vector: no residual matvec and no norm pass (||b||
// is already known), and the solution update overwrites x.
static aao_status b_gmres(aao_batch b, const double *bvec, double *x, int m, double tol, int maxit,
                          aao_info *infos, int transpose, bool zero = false)
{
    if (m < 1 || m > kBMaxRestart) {
        b->err = "restart must be in [1, 63]";
        return AAO_ERR_ARG;
    }
    if (!bvec || !x || !(tol >= 0.0) || maxit < 0) {
        b->err = "bad arguments";
        return AAO_ERR_ARG;
    }
    if (b_overlap(b, bvec, x)) {
        b->err = "b and x overlap";
        return AAO_ERR_ARG;
    }
    BT(ensure_ws(b, m));
    const size_t N = b->Ntot;
    const int P = b->count;
    BState &s = b->bs;
    s.maxit = maxit;
    const BatchLaunch Lall = b->launch(false);
    // reset state: iters, flags, fail flag (fill kernels would do for capture; this
    // part is not captured)
    BH(hipMemsetAsync(b->iv, 0, sizeof(int) * (2 * P + 1), b->st));
    BH(hipMemsetAsync(b->flags, 0, 3 * P, b->st));
    BH(hipMemsetAsync(b->fail, 0, sizeof(int), b->st));
    // ||b_p||
    const double *bp[1] = {bvec};
    BH(hipMemcpyAsync(b->dB, bp, sizeof(double *), hipMemcpyHostToDevice, b->st));
    BH(batch_cgs(0, Lall, b->dB, 1, bvec, nullptr, 0, nullptr, b->part, b->ldp, false, b->st));
    BH(batch_reduce(Lall, b->part, b->ldp, 1, s.dsum, s.sst, false, b->st));
    std::vector<double> hd((size_t)P * s.sst);
    BH(hipMemcpyAsync(hd.data(), s.dsum, sizeof(double) * hd.size(), hipMemcpyDeviceToHost, b->st));
    BH(hipStreamSynchronize(b->st));
    std::vector<double> bn(P);
    for (int p = 0; p < P; ++p) bn[p] = std::sqrt(hd[(size_t)p * s.sst]);
    for (int p = 0; p < P; ++p)
        if (!std::isfinite(bn[p])) {
            b->err = "non-finite right-hand side";
            return AAO_ERR_NUMERIC;
        }
    // zero right-hand sides: x = 0 and done (bnorm 1 avoids 0/0 in the state)
    std::vector<double> bn_dev(P);
    for (int p = 0; p < P; ++p) bn_dev[p] = bn[p] > 0.0 ? bn[p] : 1.0;
    BH(hipMemcpy(s.bnorm, bn_dev.data(), sizeof(double) * P, hipMemcpyHostToDevice));

    if (b->graph_m != m || b->graph_tol != tol || b->graph_maxit != maxit ||
        b->graph_transpose != transpose || b->graph_delayed != (int)b->delayed ||
        b->graph_span != b->span || (int)b->graphs.size() != m) {
        for (auto g : b->graphs)
            if (g) (void)hipGraphExecDestroy(g);
        b->graphs.assign(m, nullptr);
        b->graph_m = m;
        b->graph_tol = tol;
        b->graph_maxit = maxit;
        b->graph_transpose = transpose;
        b->graph_delayed = (int)b->delayed;
        b->graph_span = b->span;
    }
    int nact = 0;
    int cycles = 0;
    while (true) {
        // r = b - A x -> V_0, beta_p, vs_0, g_0, active/done
        const bool from_b = zero && cycles == 0;
        if (from_b) {
            // V_0 = b: the pointer table's first entry names b for this cycle (the
            // steps read V_0 through it); dsum still holds ||b_p||^2
            b->first_b = bvec;
            BH(hipMemcpyAsync(b->dV, &b->first_b, sizeof(double *), hipMemcpyHostToDevice,
                              b->st));
        } else {
            // the matvec leaves the tile partials of |b - A x|^2
            BH(batch_matvec(Lall, x, b->V, bvec, b->scheme, transpose, false, b->st, nullptr, -1,
                            b->part, b->ldp));
            BH(batch_reduce(Lall, b->part, b->ldp, 1, s.dsum, s.sst, false, b->st, Lall.mranges));
        }
        BH(batch_small(3, P, 0, m, tol, s, b->st));
        BH(batch_count_active(s.active, P, b->iv + 2 * P, b->st));
        BH(hipMemcpyAsync(&nact, b->iv + 2 * P, sizeof(int), hipMemcpyDeviceToHost, b->st));
        BH(hipStreamSynchronize(b->st));
        if (nact == 0) {
            if (from_b) {
                // every b_p already meets tol (or is zero): x = 0
                BH(hipMemsetAsync(x, 0, sizeof(double) * N, b->st));
                b->first_v = b->V;
                BH(hipMemcpyAsync(b->dV, &b->first_v, sizeof(double *), hipMemcpyHostToDevice,
                                  b->st));
            }
            break;
        }
        // Arnoldi steps in groups of `span` (the rest of the cycle when span = 0), each
        // group one captured graph; the host reads the number of active problems once per
        // group.  Steps after every problem has converged run fully masked (each kernel
        // finds no active work and returns), so a group's result does not depend on where
        // the groups end.
        int steps_run = 0;
        for (int j = 0; j < m;) {
            if (from_b && j == 0) {
                // the captured steps read V_0 from the workspace: step 0 of a cycle that
                // starts from b is launched eagerly
                BT(b_step(b, 0, m, tol, transpose, bvec));
                j = 1;
            } else {
                const int j1 = b->span <= 0 ? m : std::min(m, j + b->span);
                if (b->use_graph && b->st) {
                    if (!b->graphs[j]) {
                        hipGraph_t g = nullptr;
                        BH(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
                        aao_status cs = AAO_OK;
                        for (int q = j; q < j1 && cs == AAO_OK; ++q) cs = b_step(b, q, m, tol, transpose);
                        hipError_t ce = hipStreamEndCapture(b->st, &g);
                        if (cs < 0) return cs;
                        BH(ce);
                        BH(hipGraphInstantiate(&b->graphs[j], g, nullptr, nullptr, 0));
                        (void)hipGraphDestroy(g);
                    }
                    BH(hipGraphLaunch(b->graphs[j], b->st));
                } else {
                    for (int q = j; q < j1; ++q) BT(b_step(b, q, m, tol, transpose));
                }
                j = j1;
            }
            steps_run = j;
            BH(hipMemcpyAsync(&nact, b->iv + 2 * P, sizeof(int), hipMemcpyDeviceToHost, b->st));
            BH(hipStreamSynchronize(b->st));
            if (nact == 0) break;
        }
        BH(batch_backsolve(P, m, s, b->st));
        BH(batch_axpy(Lall, b->dZ, s, x, from_b, b->st, steps_run));
        if (from_b) {
            b->first_v = b->V;
            BH(hipMemcpyAsync(b->dV, &b->first_v, sizeof(double *), hipMemcpyHostToDevice, b->st));
        }
        ++cycles;
    }
    // report
    std::vector<int> it(P);
    std::vector<unsigned char> done(P), bad(P);
    std::vector<double> est(P), tr(P);
    BH(hipMemcpy(it.data(), s.iters, sizeof(int) * P, hipMemcpyDeviceToHost));
    BH(hipMemcpy(done.data(), s.done, P, hipMemcpyDeviceToHost));
    BH(hipMemcpy(bad.data(), s.bad, P, hipMemcpyDeviceToHost));
    BH(hipMemcpy(est.data(), s.est, sizeof(double) * P, hipMemcpyDeviceToHost));
    BH(hipMemcpy(tr.data(), s.truer, sizeof(double) * P, hipMemcpyDeviceToHost));
    int failed = 0;
    BH(hipMemcpy(&failed, b->fail, sizeof(int), hipMemcpyDeviceToHost));
    bool all = true, anybad = failed != 0;
    for (int p = 0; p < P; ++p) {
        if (infos) {
            infos[p].iters = it[p];
            infos[p].restarts = std::max(0, cycles - 1);
            infos[p].converged = done[p] ? 1 : 0;
            infos[p].rel_resid_est = bn[p] > 0.0 ? est[p] : 0.0;
            infos[p].rel_resid_true = bn[p] > 0.0 ? tr[p] : 0.0;
        }
        all = all && done[p];
        anybad = anybad || bad[p];
    }
    if (anybad) {
        b->err = "numerical breakdown in a batch member";
        return AAO_ERR_NUMERIC;
    }
    return all ? AAO_OK : AAO_NOT_CONVERGED;
}

// candidates of each batch launch-shape kind
static std::vector<int> bcfg_candidates(int kind)
{
    if (kind == AAO_BCFG_SLAB) return {1024, 2048, 4096, 8192, 16384};
    if (kind == AAO_BCFG_MATVEC_ROWS) return {2, 4, 8};
    return {1, 2, 4, 0};
}

static bool bcfg_ok(int kind, int value)
{
    if (kind == AAO_BCFG_SLAB) return value >= 256 && value <= 65536 && (value & (value - 1)) == 0;
    if (kind == AAO_BCFG_MATVEC_ROWS) return value == 2 || value == 4 || value == 8;
    if (kind == AAO_BCFG_GRAPH_SPAN) return value >= 0 && value <= kBMaxRestart;
    return false;
}

static aao_status bcfg_apply(aao_batch b, int kind, int value)
{
    if (kind == AAO_BCFG_GRAPH_SPAN) {
        b->span = value;   // the graph set is rebuilt by the next solve
        return AAO_OK;
    }
    if (kind == AAO_BCFG_SLAB) {
        if (b->slab == value) return AAO_OK;
        b->slab = value;
    } else {
        if (b->mrows == value) return AAO_OK;
        b->mrows = value;
    }
    BH(hipStreamSynchronize(b->st));
    return build_work_tables(b);
}

// a key of the member sizes for the tuning cache
static int64_t batch_hash(const aao_batch b)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix((uint64_t)b->scheme);
    for (const BProb &q : b->hp) {
        mix((uint64_t)q.n);
        mix((uint64_t)q.ell);
    }
    return (int64_t)(h >> 1);
}

// time `reps` calls of fn on the batch stream (ms per call)
template <typename F>
static aao_status btime(aao_batch b, int reps, F fn, double *ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BH(hipEventCreate(&e0));
    BH(hipEventCreate(&e1));
    aao_status s = fn();   // warm-up
    if (s == AAO_OK && hipEventRecord(e0, b->st) != hipSuccess) s = AAO_ERR_HIP;
    for (int r = 0; r < reps && s == AAO_OK; ++r) s = fn();
    float t = 0.0f;
    if (s == AAO_OK && (hipEventRecord(e1, b->st) != hipSuccess ||
                        hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        s = AAO_ERR_HIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / reps;
    return s;
}

// ------------------------------------------------------------------- ABI

extern "C" {

aao_status aao_batch_create(int count, const int64_t *n, const int64_t *ell, const double *tau,
                            const double *kappa, int scheme, int prec, aao_batch *out)
{
    if (!out) return AAO_ERR_ARG;
    *out = nullptr;
    if (count < 1 || !n || !ell || !kappa) return AAO_ERR_ARG;
    if (scheme != AAO_HEAT_IE && scheme != AAO_WAVE_BD2) return AAO_ERR_ARG;
    if (prec != AAO_PREC_FP64 && prec != AAO_PREC_MIXED && prec != AAO_PREC_FP32 &&
        prec != AAO_PREC_MIXED_IN)
        return AAO_ERR_ARG;
    for (int p = 0; p < count; ++p) {
        const double tp = tau ? tau[p] : 1.0 / (double)ell[p];
        if (n[p] < 1 || ell[p] < 2 || !(tp > 0.0) || !(kappa[p] > 0.0)) return AAO_ERR_ARG;
        if (n[p] > 4096 || ell[p] > 2048) return AAO_ERR_UNSUPPORTED;
    }
    aao_batch b = nullptr;
    try {
        b = new aao_batch_s();
    } catch (...) {
        return AAO_ERR_ALLOC;
    }
    b->count = count;
    b->scheme = scheme;
    b->prec = prec;
    aao_status s = AAO_OK;
    do {
        std::vector<int2> ft, rw;
        std::vector<int2> rwc[kSolveClasses];   // spectrum rows by class of n
        size_t off = 0, soff = 0, coff = 0, boff = 0;
        int max_ell = 0, max_M = 0;
        for (int p = 0; p < count; ++p) {
            BProb q{};
            q.n = (int)n[p];
            q.ell = (int)ell[p];
            q.lds = (q.n + 15) / 16 * 16;
            int M = 512;
            while (M < 2 * q.ell - 1) M *= 2;
            q.M = M;
            q.tau = tau ? tau[p] : 1.0 / (double)q.ell;
            q.kappa = kappa[p];
            q.off = (long long)off;
            q.soff = (long long)soff;
            q.coff = (long long)coff;
            q.boff = (long long)boff;
            const size_t Np = (size_t)q.n * q.ell;
            off += (Np + 63) / 64 * 64;
            soff += (size_t)(q.ell / 2 + 1) * q.lds;
            coff += q.ell;
            boff += 2 * (size_t)M;
            max_ell = std::max(max_ell, q.ell);
            max_M = std::max(max_M, M);
            b->hp.push_back(q);
            const int Wp = bluestein_pairs(M);                 // column pairs per transform tile
            const int ntile = (q.n + 2 * Wp - 1) / (2 * Wp);
            for (int t = 0; t < ntile; ++t) ft.push_back({p, t});
            for (int j = 0; j <= q.ell / 2; ++j) rwc[solve_class(q.n)].push_back({p, j});
        }
        b->Ntot = off;
        b->Stot = soff;
        b->nftiles = (int)ft.size();
        b->row_start[0] = 0;
        for (int c = 0; c < kSolveClasses; ++c) {
            rw.insert(rw.end(), rwc[c].begin(), rwc[c].end());
            b->row_start[c + 1] = (int)rw.size();
        }
        b->nrows = (int)rw.size();
        if ((s = upload(b, &b->probs, b->hp)) != AAO_OK) break;
        if ((s = upload(b, &b->ftiles, ft)) != AAO_OK) break;
        if ((s = upload(b, &b->rows, rw)) != AAO_OK) break;
        if ((s = build_work_tables(b)) != AAO_OK) break;
        if ((s = balloc(b, (void **)&b->chirp, sizeof(double) * 2 * coff)) != AAO_OK) break;
        if ((s = balloc(b, (void **)&b->bhat, sizeof(double) * 2 * boff)) != AAO_OK) break;
        if ((s = balloc(b, (void **)&b->tw, sizeof(double) * 2 * 4096)) != AAO_OK) break;
        if ((s = balloc(b, &b->spec, sizeof(double) * 2 * soff)) != AAO_OK) break;
        if (prec == AAO_PREC_MIXED_IN &&
            (s = balloc(b, &b->spec_in, sizeof(float) * 2 * soff)) != AAO_OK)
            break;
        if ((s = balloc(b, (void **)&b->fail, sizeof(int))) != AAO_OK) break;
        // small per-problem arrays: 10 arrays of kBSmall doubles + 3 scalars per problem
        const size_t smn = (size_t)count * kBSmall;
        if ((s = balloc(b, (void **)&b->sm, sizeof(double) * (10 * smn + 3 * (size_t)count))) != AAO_OK) break;
        if ((s = balloc(b, (void **)&b->H, sizeof(double) * (size_t)count * (kBMaxRestart + 1) * kBMaxRestart)) != AAO_OK) break;
        if ((s = balloc(b, (void **)&b->iv, sizeof(int) * (2 * count + 1))) != AAO_OK) break;
        if ((s = balloc(b, (void **)&b->flags, 3 * (size_t)count)) != AAO_OK) break;
        if ((s = balloc(b, (void **)&b->dB, sizeof(double *))) != AAO_OK) break;
        BState &bs = b->bs;
        bs.sst = kBSmall;
        bs.hst = (long long)(kBMaxRestart + 1) * kBMaxRestart;
        bs.dsum = b->sm;
        bs.h1 = b->sm + smn;
        bs.h2 = b->sm + 2 * smn;
        bs.coef = b->sm + 3 * smn;
        bs.vs = b->sm + 4 * smn;
        bs.cs = b->sm + 5 * smn;
        bs.sn = b->sm + 6 * smn;
        bs.g = b->sm + 7 * smn;
        bs.y = b->sm + 8 * smn;
        bs.bnorm = b->sm + 10 * smn;
        bs.est = bs.bnorm + count;
        bs.truer = bs.est + count;
        bs.H = b->H;
        bs.iters = b->iv;
        bs.ksteps = b->iv + count;
        bs.active = b->flags;
        bs.done = b->flags + count;
        bs.bad = b->flags + 2 * count;
        if (hipStreamCreate(&b->st) != hipSuccess) {
            s = AAO_ERR_HIP;
            break;
        }
        b->own_stream = true;
        if (batch_prepare() != hipSuccess ||
            hipMemset(b->sm, 0, sizeof(double) * (10 * smn + 3 * (size_t)count)) != hipSuccess ||
            launch_twiddles(b->tw, 4096, 4096, b->st) != hipSuccess ||
            batch_setup_tables(b->probs, count, max_ell, max_M, b->chirp, b->bhat, b->st) != hipSuccess ||
            hipStreamSynchronize(b->st) != hipSuccess) {
            s = AAO_ERR_HIP;
            break;
        }
    } while (0);
    if (s != AAO_OK) {
        aao_batch_destroy(b);
        return s;
    }
    *out = b;
    return AAO_OK;
}

aao_status aao_batch_destroy(aao_batch b)
{
    if (!b) return AAO_OK;
    if (b->st) (void)hipStreamSynchronize(b->st);
    free_ws(b);
    (void)hipFree(b->probs);
    (void)hipFree(b->ftiles);
    (void)hipFree(b->rows);
    (void)hipFree(b->mtiles);
    (void)hipFree(b->slabs);
    (void)hipFree(b->pslabs);
    (void)hipFree(b->mranges);
    (void)hipFree(b->chirp);
    (void)hipFree(b->bhat);
    (void)hipFree(b->tw);
    (void)hipFree(b->spec);
    (void)hipFree(b->spec_in);
    (void)hipFree(b->fail);
    (void)hipFree(b->part);
    (void)hipFree(b->sm);
    (void)hipFree(b->H);
    (void)hipFree(b->iv);
    (void)hipFree(b->flags);
    (void)hipFree(b->dB);
    if (b->own_stream && b->st) (void)hipStreamDestroy(b->st);
    delete b;
    return AAO_OK;
}

aao_status aao_batch_offsets(aao_batch b, int64_t *offsets, int64_t *total)
{
    if (!b) return AAO_ERR_ARG;
    if (offsets)
        for (int p = 0; p < b->count; ++p) offsets[p] = b->hp[p].off;
    if (total) *total = (int64_t)b->Ntot;
    return AAO_OK;
}

aao_status aao_batch_set_graph(aao_batch b, int enable)
{
    if (!b) return AAO_ERR_ARG;
    b->use_graph = enable != 0;
    return AAO_OK;
}

aao_status aao_batch_get_config(aao_batch b, int kind, int *value)
{
    if (!b || !value || kind < 0 || kind >= AAO_NUM_BCFG) return AAO_ERR_ARG;
    *value = kind == AAO_BCFG_SLAB ? b->slab : kind == AAO_BCFG_MATVEC_ROWS ? b->mrows : b->span;
    return AAO_OK;
}

aao_status aao_batch_set_config(aao_batch b, int kind, int value)
{
    if (!b || kind < 0 || kind >= AAO_NUM_BCFG) return AAO_ERR_ARG;
    if (b->broken) return AAO_ERR_HIP;
    if (!bcfg_ok(kind, value)) {
        b->err = "launch shape out of range";
        return AAO_ERR_ARG;
    }
    return bcfg_apply(b, kind, value);
}

aao_status aao_batch_tune(aao_batch b, const double *bvec, int restart, double tol, int maxit,
                          int reps)
{
    if (!b) return AAO_ERR_ARG;
    if (b->broken) return AAO_ERR_HIP;
    if (reps < 1 || reps > 100 || (bvec && (restart < 1 || restart > kBMaxRestart))) {
        b->err = "bad tuning arguments";
        return AAO_ERR_ARG;
    }
    int device = 0;
    BH(hipGetDevice(&device));
    const int64_t key = batch_hash(b);
    // scratch: a 4-vector basis, search directions and w (the workspace), x for the solves
    try {
        BT(ensure_ws(b, std::max(4, bvec ? restart : 4)));
        const size_t N = b->Ntot;
        BH(launch_fill(b->V, 0.0, N * (b->m_alloc + 1), b->st));
        BH(launch_fill(b->W, 0.0, N, b->st));
        for (int kind = 0; kind < AAO_NUM_BCFG; ++kind) {
            if (kind == AAO_BCFG_GRAPH_SPAN && !bvec) continue;
            int code = 0;
            if (tune_cache_get(device, 100 + kind, b->prec, b->count, key, &code) &&
                bcfg_ok(kind, code)) {
                BT(bcfg_apply(b, kind, code));
                continue;
            }
            int best = -1;
            double best_ms = 0.0;
            double *xs = nullptr;
            if (kind == AAO_BCFG_GRAPH_SPAN) BT(balloc(b, (void **)&xs, sizeof(double) * N));
            for (int v : bcfg_candidates(kind)) {
                aao_status st = bcfg_apply(b, kind, v);
                double ms = 0.0;
                const BatchLaunch L = b->launch(false);
                if (st == AAO_OK && kind == AAO_BCFG_SLAB) {
                    // the slab passes: an update with four basis vectors and their dots
                    st = btime(b, reps, [&]() -> aao_status {
                        BH(batch_cgs(1, L, b->dV, 4, b->W, b->bs.coef, b->bs.sst, nullptr,
                                     b->part, b->ldp, false, b->st));
                        BH(batch_reduce(L, b->part, b->ldp, 4, b->bs.dsum, b->bs.sst, false,
                                        b->st));
                        return AAO_OK;
                    }, &ms);
                } else if (st == AAO_OK && kind == AAO_BCFG_MATVEC_ROWS) {
                    // a plain matvec and one that forms two Gram-Schmidt dots
                    st = btime(b, reps, [&]() -> aao_status {
                        BH(batch_matvec(L, b->V, b->W, nullptr, b->scheme, 0, false, b->st));
                        BH(batch_matvec(L, b->V + N, b->W, nullptr, b->scheme, 0, false, b->st,
                                        b->dV, 2, b->part, b->ldp));
                        return AAO_OK;
                    }, &ms);
                } else if (st == AAO_OK) {
                    st = btime(b, reps, [&]() -> aao_status {
                        const aao_status r = b_gmres(b, bvec, xs, restart, tol, maxit, nullptr,
                                                     0, true);
                        return r < 0 ? r : AAO_OK;
                    }, &ms);
                }
                if (st != AAO_OK) {
                    (void)hipFree(xs);
                    return st;
                }
                if (best < 0 || ms < best_ms) {
                    best = v;
                    best_ms = ms;
                }
            }
            (void)hipFree(xs);
            BT(bcfg_apply(b, kind, best));
            tune_cache_put(device, 100 + kind, b->prec, b->count, key, best, 1e3 * best_ms);
        }
    } catch (...) {
        return AAO_ERR_ALLOC;
    }
    BH(hipStreamSynchronize(b->st));
    return AAO_OK;
}

aao_status aao_batch_apply_A(aao_batch b, const double *x, double *y, int transpose)
{
    if (!b) return AAO_ERR_ARG;
    if (b->broken) return AAO_ERR_HIP;
    if (!x || !y) return AAO_ERR_ARG;
    if (b_overlap(b, x, y)) {
        b->err = "x and y overlap";
        return AAO_ERR_ARG;
    }
    BH(batch_matvec(b->launch(false), x, y, nullptr, b->scheme, transpose ? 1 : 0, false, b->st));
    BH(hipStreamSynchronize(b->st));
    return AAO_OK;
}

aao_status aao_batch_apply_Pinv(aao_batch b, const double *r, double *z, int transpose)
{
    if (!b) return AAO_ERR_ARG;
    if (b->broken) return AAO_ERR_HIP;
    if (!r || !z) return AAO_ERR_ARG;
    if (b_overlap(b, r, z)) {
        b->err = "r and z overlap";
        return AAO_ERR_ARG;
    }
    BT(b_pinv(b, r, nullptr, 0, z, false, transpose ? 1 : 0));
    BH(hipStreamSynchronize(b->st));
    return AAO_OK;
}

aao_status aao_batch_gmres(aao_batch b, const double *bvec, double *x, int restart, double tol,
                           int maxit, aao_info *infos)
{
    if (!b) return AAO_ERR_ARG;
    if (b->broken) return AAO_ERR_HIP;
    try {
        return b_gmres(b, bvec, x, restart, tol, maxit, infos, 0);
    } catch (...) {
        return AAO_ERR_ALLOC;
    }
}

aao_status aao_batch_gmres_ex(aao_batch b, const double *bvec, double *x, int restart, double tol,
                              int maxit, int flags, aao_info *infos)
{
    if (!b) return AAO_ERR_ARG;
    if (b->broken) return AAO_ERR_HIP;
    if (flags & ~(AAO_GMRES_ZERO_GUESS | AAO_GMRES_TRANSPOSE | AAO_GMRES_CGS2_CLASSIC)) {
        b->err = "unknown flag bits";
        return AAO_ERR_ARG;
    }
    b->delayed = (flags & AAO_GMRES_CGS2_CLASSIC) == 0;
    try {
        return b_gmres(b, bvec, x, restart, tol, maxit, infos,
                       (flags & AAO_GMRES_TRANSPOSE) ? 1 : 0, (flags & AAO_GMRES_ZERO_GUESS) != 0);
    } catch (...) {
        return AAO_ERR_ALLOC;
    }
}

aao_status aao_batch_project_sine(aao_batch b, int J, const int *modes, const double *amps,
                                  double *u0)
{
    if (!b) return AAO_ERR_ARG;
    if (b->broken) return AAO_ERR_HIP;
    if (J < 1 || !modes || !amps || !u0) return AAO_ERR_ARG;
    for (int q = 0; q < J; ++q)
        if (modes[q] < 1) return AAO_ERR_ARG;
    int *dm = nullptr;
    double *da = nullptr;
    BT(balloc(b, (void **)&dm, sizeof(int) * J));
    aao_status s = balloc(b, (void **)&da, sizeof(double) * (size_t)J * b->count);
    if (s != AAO_OK) {
        (void)hipFree(dm);
        return s;
    }
    hipError_t e = hipMemcpy(dm, modes, sizeof(int) * J, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(da, amps, sizeof(double) * (size_t)J * b->count, hipMemcpyHostToDevice);
    size_t uoff = 0;
    for (int p = 0; p < b->count && e == hipSuccess; ++p) {
        e = launch_project_sine(u0 + uoff, b->hp[p].n, J, dm, da + (size_t)p * J, b->st);
        uoff += b->hp[p].n;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    (void)hipFree(dm);
    (void)hipFree(da);
    BH(e);
    return AAO_OK;
}

aao_status aao_batch_build_rhs(aao_batch b, const double *u0, double *bvec)
{
    if (!b) return AAO_ERR_ARG;
    if (b->broken) return AAO_ERR_HIP;
    if (!u0 || !bvec) return AAO_ERR_ARG;
    BH(launch_fill(bvec, 0.0, b->Ntot, b->st));
    size_t uoff = 0;
    for (int p = 0; p < b->count; ++p) {
        const BProb &q = b->hp[p];
        Scheme sc{};
        if (b->scheme == AAO_HEAT_IE) {
            sc.s = 1; sc.a[0] = 1.0; sc.a[1] = -1.0; sc.b[0] = q.tau;
        } else {
            sc.s = 2; sc.a[0] = 1.0; sc.a[1] = -2.0; sc.a[2] = 1.0; sc.b[0] = q.tau * q.tau;
        }
        BH(launch_build_rhs(bvec + q.off, u0 + uoff, nullptr, q.n, q.ell, sc, q.kappa, q.tau, b->st));
        uoff += q.n;
    }
    BH(hipStreamSynchronize(b->st));
    return AAO_OK;
}

const char *aao_batch_last_error(aao_batch b) { return b ? b->err.c_str() : ""; }

}  // extern "C"
