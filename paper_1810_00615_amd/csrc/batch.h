// Device-side description of a batch of independent all-at-once problems and
// the launchers of the batched kernels (k_batch.hip).
#pragma once
#include "aao_internal.h"

#ifndef BL_THREADS_DEFAULT
#define BL_THREADS_DEFAULT 512
#endif

namespace aao {

struct BProb {
    int n, ell, lds, M;          // M: Bluestein convolution length, power of two >= 2 ell - 1
    double tau, kappa;
    long long off;               // first element of the problem in a batch vector
    long long soff;              // first complex element of its half spectrum
    long long coff;              // first entry of its chirp table (ell entries)
    long long boff;              // first entry of its filter spectra (2 M entries)
};

// Per-problem GMRES state (device arrays; `sst` doubles per problem for the
// small vectors, `hst` for the Hessenberg matrix, column-major (m+1) x m).
struct BState {
    int sst;
    long long hst;
    int maxit;
    double *dsum, *h1, *h2, *coef, *vs, *H, *cs, *sn, *g, *y, *bnorm, *est, *truer;
    int *iters, *ksteps;
    unsigned char *active, *done, *bad;
};

// Work tables of one batch (device pointers).
struct BatchLaunch {
    const BProb *probs;
    int count;
    const int2 *ftiles;  int nftiles;   // transform tiles (problem, tile)
    const int2 *rows;    int nrows;     // spectrum rows (problem, frequency), by class of n
    int row_start[5];                   // rows of class c: [row_start[c], row_start[c + 1])
    const int4 *mtiles;  int nmtiles;   // matvec tiles (problem, column block, row block, -)
    int mrows;                          // time levels per matvec tile (2, 4 or 8)
    const int4 *slabs;   int nslabs;    // element slabs (problem, first, count, -)
    const int2 *pslabs;                 // slab range [x, y) of every problem
    const int2 *mranges;                // matvec tile range [x, y) of every problem
    const unsigned char *active;        // per-problem mask
    const double *chirp, *bhat, *tw;    // Bluestein tables, 4096-point twiddles
};

// launch shapes of a batch (aao_batch_tune / aao_batch_set_config): elements per
// Gram-Schmidt / update slab, time levels per matvec tile, Arnoldi steps per graph
constexpr int kBatchSlabDefault = 4096;
constexpr int kMatvecRowsDefault = 4;
constexpr int kGraphSpanDefault = 1;
constexpr int kBSmall = 72;             // doubles per problem in the small per-problem arrays
// shifted solves: class c = 0..3 of a problem holds n <= 8 * (64 << c) (workgroups of
// 64 << c threads, 8 unknowns per thread)
constexpr int kSolveClasses = 4;
constexpr int solve_class(int n) { return n <= 512 ? 0 : n <= 1024 ? 1 : n <= 2048 ? 2 : 3; }
// Bluestein transforms: points per thread of the length-M FFTs and threads per
// workgroup; a workgroup transforms kBluesteinThreads P / M column pairs
constexpr int kBluesteinP = 8;
constexpr int kBluesteinThreads = BL_THREADS_DEFAULT;
constexpr int bluestein_pairs(int M) { return kBluesteinThreads * kBluesteinP / M; }

hipError_t batch_prepare();
hipError_t batch_setup_tables(const BProb *probs, int count, int max_ell, int max_M,
                              double *chirp, double *bhat, hipStream_t st);
hipError_t batch_fft_fwd(const BatchLaunch &L, const double *r, const double *scales, int sstride,
                         void *spec, bool single, hipStream_t st);
hipError_t batch_fft_inv(const BatchLaunch &L, const void *spec, double *z, bool single,
                         hipStream_t st);
// right-hand sides from `in`, solutions to `out` (in place when in == out); element
// types float2 / double2 by single_in / single_out, arithmetic by single_arith
hipError_t batch_solve(const BatchLaunch &L, const void *in, void *out, bool single_in,
                       bool single_out, bool single_arith, int scheme, int transpose, int *fail,
                       hipStream_t st);
// nd = 1..4: the tiles also leave the partials of Vd[q] . y (q < nd) at
// part[tile * ldp + q] (reduced per problem over L.mranges); nd = -1: the partial
// of y . y at part[tile * ldp]
hipError_t batch_matvec(const BatchLaunch &L, const double *x, double *y, const double *bsub,
                        int scheme, int transpose, bool masked, hipStream_t st,
                        const double *const *Vd = nullptr, int nd = 0, double *part = nullptr,
                        int ldp = 0);
hipError_t batch_cgs(int mode, const BatchLaunch &L, const double *const *V, int nv,
                     const double *w, const double *coef, int cst, double *out, double *part,
                     int ldp, bool masked, hipStream_t st);
// The deferred-re-orthogonalisation update of step nv - 1 (coefficients from
// batch_small mode 4): v_j written over the pending vector (j > 0), w1 to out,
// partials V_i . w1, v_j . w1, w1 . w1 (nv + 1 slots)
hipError_t batch_cgs_delayed(const BatchLaunch &L, const double *const *V, int nv,
                             const double *w, const BState &s, double *out, double *part, int ldp,
                             hipStream_t st);
// ranges: per-problem block ranges of part (L.pslabs when null)
hipError_t batch_reduce(const BatchLaunch &L, const double *part, int ldp, int cnt, double *sums,
                        int sst, bool masked, hipStream_t st, const int2 *ranges = nullptr);
hipError_t batch_small(int mode, int count, int j, int m, double tol, const BState &s,
                       hipStream_t st);
hipError_t batch_backsolve(int count, int m, const BState &s, hipStream_t st);
// kmax: an upper bound of every problem's step count in the cycle (<= 64)
hipError_t batch_axpy(const BatchLaunch &L, const double *const *Z, const BState &s, double *x,
                      bool overwrite, hipStream_t st, int kmax);
hipError_t batch_count_active(const unsigned char *a, int count, int *nact, hipStream_t st);

}  // namespace aao
