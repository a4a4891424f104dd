/*
 * Reference oracle for the all-at-once (monolithic) time-stepping systems of
 * Goddard & Wathen, "A note on parallel preconditioning for all-at-once
 * evolutionary PDEs" (arXiv 1810.00615), and of the block-circulant
 * preconditioner of McDonald, Pestana & Wathen that it parallelises.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU statement of what the GPU library computes.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant with the GPU library.
 *
 * Everything is IEEE double precision, straight loops, no blocking or fusion.
 * OpenMP is used only to run independent units (columns, frequencies) at once.
 *
 * Conventions (the paper's readings are listed in the design notes):
 *   - n interior nodes of a uniform P1 mesh on [0,1], h = 1/(n+1)         (Sec. 2)
 *   - M = (h/6) tridiag(1,4,1), K = (1/h) tridiag(-1,2,-1)  (standard Galerkin,
 *     Sec. 2, eq. applyEuler); the diffusivity kappa multiplies K.
 *   - a vector of the monolithic system is ell x n, row k = time level k+1,
 *     row-major (the ordering [u_1; ...; u_ell] of eq. monolithicheat).
 *   - the block in row k, column k - m of the monolithic matrix is
 *     a_m M + b_m kappa K (or_block); Toeplitz schemes use the same pair on every row:
 *       heat, implicit Euler (eq. timestepproblem1, read as M + tau K):
 *             A_0 = M + tau kappa K, A_1 = -M
 *       wave, BD2 (eq. BD2 and the system C_BD2):
 *             A_0 = M + tau^2 kappa K, A_1 = -2M, A_2 = M
 *       wave, BD4 (eq. BD4 and the system C_BD4): A_0 = 2M + tau^2 kappa K,
 *             A_1 = -5M, A_2 = 4M, A_3 = -M from the third row on; the first two rows
 *             are the start-up rows B u_1 and C u_1 + B u_2, B = M + tau^2 kappa K,
 *             C = -2M (not Toeplitz)
 *       wave, central differences (eq. CenDiffDisc and the system C_CD): two-sided,
 *             M u_{k-1} + (tau^2 kappa K - 2M) u_k + M u_{k+1}, i.e. offsets
 *             m = -1, 0, 1 (the last row has no u_{ell+1}); its exact solve is the
 *             banded elimination in oracle/__init__.py
 *   - the DFT along time is X_j = sum_k x_k w^{jk}, w = exp(-2 pi i/ell).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_HEAT 0
#define OR_BD2 1
#define OR_BD4 2
#define OR_CD 3

/* ---------------------------------------------------------------- scheme */

/* Toeplitz coefficients (a_m, b_m) of the scheme for offsets m = mlo..mhi (entry
 * m - mlo): the blocks a_m M + b_m kappa K of every row away from the start-up rows,
 * and so the blocks of the circulant preconditioner.
 *   heat: eq. monolithicheat (A_0 = M + tau K after the implicit Euler step, A_1 = -M)
 *   BD2:  the system C_BD2 (A_0 = M + tau^2 K, A_1 = -2M, A_2 = M)
 *   BD4:  the system C_BD4 (A_0 = 2M + tau^2 K, A_1 = -5M, A_2 = 4M, A_3 = -M)
 *   CD:   the system C_CD (M below, tau^2 K - 2M on, M above the diagonal)
 * Returns 0, or -1 for an unknown scheme. */
int or_toeplitz(int scheme, double tau, int *mlo, int *mhi, double *a, double *b)
{
    const double t2 = tau * tau;
    switch (scheme) {
    case OR_HEAT:
        *mlo = 0; *mhi = 1;
        a[0] = 1.0;  b[0] = tau;
        a[1] = -1.0; b[1] = 0.0;
        return 0;
    case OR_BD2:
        *mlo = 0; *mhi = 2;
        a[0] = 1.0;  b[0] = t2;
        a[1] = -2.0; b[1] = 0.0;
        a[2] = 1.0;  b[2] = 0.0;
        return 0;
    case OR_BD4:
        *mlo = 0; *mhi = 3;
        a[0] = 2.0;  b[0] = t2;
        a[1] = -5.0; b[1] = 0.0;
        a[2] = 4.0;  b[2] = 0.0;
        a[3] = -1.0; b[3] = 0.0;
        return 0;
    case OR_CD:
        *mlo = -1; *mhi = 1;
        a[0] = 1.0;  b[0] = 0.0;     /* m = -1: M u_{k+1} */
        a[1] = -2.0; b[1] = t2;      /* m =  0 */
        a[2] = 1.0;  b[2] = 0.0;     /* m =  1: M u_{k-1} */
        return 0;
    default:
        return -1;
    }
}

/* Lower-triangular Toeplitz schemes (heat, BD2, BD4): coefficients of offsets
 * 0..s; returns s, or -1 (unknown scheme, or a two-sided scheme). */
int or_scheme_coeffs(int scheme, double tau, double *a, double *b)
{
    int mlo, mhi;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0 || mlo != 0) return -1;
    return mhi;
}

/* The block in row k (0-based), column k - m of the monolithic matrix of size
 * ell: *cm M + *ck K.  Returns 1 if that block exists, else 0 (outside the matrix
 * or zero).  BD4 rows 0 and 1 are the start-up rows of the system C_BD4; with
 * variable steps tau_k (heat, eq. nonuniformmonolithicheat) the diagonal block of
 * row k is M + tau_k kappa K. */
int or_block(int scheme, double tau, double kappa, const double *tau_k, int ell, int k, int m,
             double *cm, double *ck)
{
    double a[4], b[4];
    int mlo, mhi;
    if (k < 0 || k >= ell || k - m < 0 || k - m >= ell) return 0;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0 || m < mlo || m > mhi) return 0;
    *cm = a[m - mlo];
    *ck = b[m - mlo] * kappa;
    if (scheme == OR_HEAT && m == 0 && tau_k) *ck = tau_k[k] * kappa;
    if (scheme == OR_BD4 && k < 2) {
        /* start-up rows: B u_1 = .., C u_1 + B u_2 = .. (BD2 steps) */
        if (m == 0) {
            *cm = 1.0;
            *ck = tau * tau * kappa;
        } else if (m == 1) {
            *cm = -2.0;
            *ck = 0.0;
        } else {
            return 0;
        }
    }
    return 1;
}

/* ------------------------------------------------------- space operators */

/* y = (cm M + ck K) x for one time level (both matrices tridiagonal; zero
 * Dirichlet values outside 0..n-1). */
static void mk_apply(int n, double cm, double ck, const double *x, double *y)
{
    double h = 1.0 / (n + 1);
    for (int i = 0; i < n; ++i) {
        double xl = (i > 0) ? x[i - 1] : 0.0;
        double xr = (i < n - 1) ? x[i + 1] : 0.0;
        double mx = (h / 6.0) * (xl + 4.0 * x[i] + xr);
        double kx = (1.0 / h) * (-xl + 2.0 * x[i] - xr);
        y[i] = cm * mx + ck * kx;
    }
}

void or_mass_apply(int n, const double *x, double *y) { mk_apply(n, 1.0, 0.0, x, y); }
void or_stiff_apply(int n, const double *x, double *y) { mk_apply(n, 0.0, 1.0, x, y); }

/* Thomas algorithm (no pivoting) for a real tridiagonal system with constant
 * sub/super diagonal e and diagonal d.  Returns 0, or -4 on a zero pivot. */
static int thomas_real_toeplitz(int n, double d, double e, const double *r, double *x)
{
    double *cp = (double *)malloc(sizeof(double) * (size_t)n);
    double *gp = (double *)malloc(sizeof(double) * (size_t)n);
    int st = 0;
    double piv = d;
    if (piv == 0.0) { st = -4; goto out; }
    cp[0] = e / piv;
    gp[0] = r[0] / piv;
    for (int i = 1; i < n; ++i) {
        piv = d - e * cp[i - 1];
        if (piv == 0.0) { st = -4; goto out; }
        cp[i] = e / piv;
        gp[i] = (r[i] - e * gp[i - 1]) / piv;
    }
    x[n - 1] = gp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = gp[i] - cp[i] * x[i + 1];
out:
    free(cp);
    free(gp);
    return st;
}

/* Solve (cm M + ck K) x = r. */
static int mk_solve(int n, double cm, double ck, const double *r, double *x)
{
    double h = 1.0 / (n + 1);
    double d = cm * (4.0 * h / 6.0) + ck * (2.0 / h);
    double e = cm * (h / 6.0) - ck * (1.0 / h);
    return thomas_real_toeplitz(n, d, e, r, x);
}

int or_mk_solve(int n, double cm, double ck, const double *r, double *x)
{
    return mk_solve(n, cm, ck, r, x);
}

/* ----------------------------------------------------------- initial data */

/* L2 load vector f_i = int_0^1 s(x) phi_i(x) dx of the sine series
 * s(x) = sum_m amps[m] sin(modes[m] pi x), with phi_i the P1 hat function at
 * x_i = i h.  For one mode the integral is exact:
 *   int sin(q pi x) phi_i dx = sin(q pi x_i) * 2 (1 - cos(q pi h)) / (h q^2 pi^2).
 * The initial state of eq. timestepproblem1 is "a projection of the initial
 * data"; it is read as the L2 projection u_0 = M^{-1} f. */
void or_load_sine(int n, int J, const int *modes, const double *amps, double *f)
{
    double h = 1.0 / (n + 1);
    for (int i = 0; i < n; ++i) f[i] = 0.0;
    for (int m = 0; m < J; ++m) {
        double q = (double)modes[m];
        double sh = sin(0.5 * q * M_PI * h);          /* 1 - cos(q pi h) = 2 sin^2(q pi h/2) */
        double g = 4.0 * sh * sh / (h * q * q * M_PI * M_PI);
        for (int i = 0; i < n; ++i) f[i] += amps[m] * g * sin(q * M_PI * (i + 1) * h);
    }
}

/* u_0 = M^{-1} f (L2 projection onto the P1 space). */
int or_project_sine(int n, int J, const int *modes, const double *amps, double *u0)
{
    double *f = (double *)malloc(sizeof(double) * (size_t)n);
    or_load_sine(n, J, modes, amps, f);
    int st = mk_solve(n, 1.0, 0.0, f, u0);
    free(f);
    return st;
}

/* Right-hand side b of the monolithic system (ell x n, all rows but the first
 * one to three are zero).
 *   heat (eq. monolithicheat): b_1 = M u_0.
 *   BD2  (system C_BD2): b_1 = A_0 (u_0 + tau v_0), b_2 = -M u_0; the first row
 *        is the start-up step u_1 = u_0 + tau v_0, which is the printed row
 *        A_0 u_1 = (M + tau^2 K) u_0 when the initial velocity v_0 is zero.
 *   BD4  (system C_BD4): b_1 = B (u_0 + tau v_0), b_2 = -M u_0, b_3 = M u_0 (the
 *        same start-up step; the u_0 terms of the second and third rows moved to
 *        the right).
 *   CD   (system C_CD): b_1 = -M u_0; the scheme takes no initial velocity (v_0 must
 *        be NULL). */
int or_build_rhs(int scheme, int n, int ell, double tau, double kappa,
                 const double *u0, const double *v0, double *b)
{
    memset(b, 0, sizeof(double) * (size_t)n * (size_t)ell);
    if (scheme == OR_HEAT) {
        or_mass_apply(n, u0, b);
        return 0;
    }
    if (scheme == OR_BD2 || scheme == OR_BD4) {
        if (ell < (scheme == OR_BD2 ? 2 : 3)) return -1;
        double *w = (double *)malloc(sizeof(double) * (size_t)n);
        for (int i = 0; i < n; ++i) w[i] = u0[i] + (v0 ? tau * v0[i] : 0.0);
        mk_apply(n, 1.0, tau * tau * kappa, w, b);   /* BD2's A_0 = BD4's B */
        mk_apply(n, -1.0, 0.0, u0, b + n);
        if (scheme == OR_BD4) mk_apply(n, 1.0, 0.0, u0, b + 2 * (size_t)n);
        free(w);
        return 0;
    }
    if (scheme == OR_CD) {
        if (v0) return -1;
        mk_apply(n, -1.0, 0.0, u0, b);
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------ monolithic matvec */

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), where A is the monolithic
 * matrix of eq. monolithicheat / C_BD2 / C_BD4 / C_CD, or the variable-step matrix
 * B of eq. nonuniformmonolithicheat when tau_k != NULL.
 * Row k: (A x)_k = sum_m A_{k,k-m} x_{k-m}; every block is symmetric, so
 * (A^T x)_k = sum_m A_{k+m,k} x_{k+m}. */
int or_apply_A(int scheme, int n, int ell, double tau, double kappa, const double *tau_k,
               const double *x, double *y, int transpose)
{
    double a[4], b[4];
    int mlo, mhi;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0) return -1;
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    memset(y, 0, sizeof(double) * (size_t)n * (size_t)ell);
    for (int k = 0; k < ell; ++k) {
        for (int m = mlo; m <= mhi; ++m) {
            double cm, ck;
            const int src = transpose ? k + m : k - m;
            const int row = transpose ? k + m : k;       /* the row holding the block */
            if (!or_block(scheme, tau, kappa, tau_k, ell, row, m, &cm, &ck)) continue;
            mk_apply(n, cm, ck, x + (size_t)src * n, t);
            for (int i = 0; i < n; ++i) y[(size_t)k * n + i] += t[i];
        }
    }
    free(t);
    return 0;
}

/* y = C x: the block circulant of eq. standardheatprecon / wavepreconditioner /
 * R_BD4 / R_CD, i.e. the Toeplitz blocks wrapped around,
 * (C x)_k = sum_m A_m x_{(k-m) mod ell}.  transpose = 1 gives C^T,
 * (C^T x)_k = sum_m A_m x_{(k+m) mod ell}. */
int or_apply_C(int scheme, int n, int ell, double tau, double kappa,
               const double *x, double *y, int transpose)
{
    double a[4], b[4];
    int mlo, mhi;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0) return -1;
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    memset(y, 0, sizeof(double) * (size_t)n * (size_t)ell);
    for (int k = 0; k < ell; ++k) {
        for (int m = mlo; m <= mhi; ++m) {
            int src = transpose ? k + m : k - m;
            src = ((src % ell) + ell) % ell;
            mk_apply(n, a[m - mlo], b[m - mlo] * kappa, x + (size_t)src * n, t);
            for (int i = 0; i < n; ++i) y[(size_t)k * n + i] += t[i];
        }
    }
    free(t);
    return 0;
}

/* y = E x with E = sigma (x) kappa K = blockdiag(sigma_k kappa K),
 * sigma_k = tau_k - tau (Sec. 2, the splitting Q = P + sigma (x) K). */
int or_apply_E(int n, int ell, double tau, double kappa, const double *tau_k,
               const double *x, double *y)
{
    for (int k = 0; k < ell; ++k)
        mk_apply(n, 0.0, (tau_k[k] - tau) * kappa, x + (size_t)k * n, y + (size_t)k * n);
    return 0;
}

/* --------------------------------------------------------- exact solves */

/* Forward block substitution: the exact solution of A U = b for the lower-triangular
 * schemes, i.e. the sequential time stepping of eq. timestepproblem1 / BD2 / BD4 that
 * the monolithic system packages:
 *   u_k = A_{k,k}^{-1} (b_k - sum_{m>=1} A_{k,k-m} u_{k-m}).
 * The two-sided central-difference system is not triangular: -1 (the Python side
 * solves it as a banded system with partial pivoting). */
int or_solve_seq(int scheme, int n, int ell, double tau, double kappa, const double *tau_k,
                 const double *bvec, double *U)
{
    double a[4], b[4];
    int mlo, mhi;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0 || mlo < 0) return -1;
    double *rhs = (double *)malloc(sizeof(double) * (size_t)n);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    int st = 0;
    for (int k = 0; k < ell && st == 0; ++k) {
        memcpy(rhs, bvec + (size_t)k * n, sizeof(double) * (size_t)n);
        double cm, ck;
        for (int m = 1; m <= mhi; ++m) {
            if (!or_block(scheme, tau, kappa, tau_k, ell, k, m, &cm, &ck)) continue;
            mk_apply(n, cm, ck, U + (size_t)(k - m) * n, t);
            for (int i = 0; i < n; ++i) rhs[i] -= t[i];
        }
        or_block(scheme, tau, kappa, tau_k, ell, k, 0, &cm, &ck);
        st = mk_solve(n, cm, ck, rhs, U + (size_t)k * n);
    }
    free(rhs);
    free(t);
    return st;
}

/* Backward block substitution: the exact solution of A^T L = g,
 * l_k = A_{k,k}^{-1} (g_k - sum_{m>=1} A_{k+m,k} l_{k+m}) (every block symmetric);
 * -1 for the two-sided central-difference system, as in or_solve_seq. */
int or_adjoint_seq(int scheme, int n, int ell, double tau, double kappa, const double *tau_k,
                   const double *g, double *L)
{
    double a[4], b[4];
    int mlo, mhi;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0 || mlo < 0) return -1;
    double *rhs = (double *)malloc(sizeof(double) * (size_t)n);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    int st = 0;
    for (int k = ell - 1; k >= 0 && st == 0; --k) {
        memcpy(rhs, g + (size_t)k * n, sizeof(double) * (size_t)n);
        double cm, ck;
        for (int m = 1; m <= mhi; ++m) {
            if (!or_block(scheme, tau, kappa, tau_k, ell, k + m, m, &cm, &ck)) continue;
            mk_apply(n, cm, ck, L + (size_t)(k + m) * n, t);
            for (int i = 0; i < n; ++i) rhs[i] -= t[i];
        }
        or_block(scheme, tau, kappa, tau_k, ell, k, 0, &cm, &ck);
        st = mk_solve(n, cm, ck, rhs, L + (size_t)k * n);
    }
    free(rhs);
    free(t);
    return st;
}

/* ------------------------------------------------- Fourier diagonalisation */

/* Direct DFT along time of every column of an ell x n complex array:
 * X_j = sum_k x_k w^{s jk}, w = exp(-2 pi i/ell), s = +1 (forward) or -1
 * (inverse, which also divides by ell).  The exponent jk is reduced mod ell in
 * integer arithmetic before the sine/cosine is taken.  O(ell^2) per column.
 * This is the (U (x) I_n) product of eq. precon2para written as the per-column
 * transform of eq. alternativecal. */
void or_dft(int ell, int n, const double *xr, const double *xi, double *Xr, double *Xi, int inverse)
{
    double sgn = inverse ? 1.0 : -1.0;
    double *cs = (double *)malloc(sizeof(double) * (size_t)ell);
    double *sn = (double *)malloc(sizeof(double) * (size_t)ell);
    for (int p = 0; p < ell; ++p) {
        cs[p] = cos(2.0 * M_PI * p / ell);
        sn[p] = sgn * sin(2.0 * M_PI * p / ell);
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < ell; ++j) {
            double sr = 0.0, si = 0.0;
            for (int k = 0; k < ell; ++k) {
                int p = (int)(((long long)j * k) % ell);
                double vr = xr[(size_t)k * n + i], vi = xi ? xi[(size_t)k * n + i] : 0.0;
                sr += vr * cs[p] - vi * sn[p];
                si += vr * sn[p] + vi * cs[p];
            }
            if (inverse) { sr /= ell; si /= ell; }
            Xr[(size_t)j * n + i] = sr;
            Xi[(size_t)j * n + i] = si;
        }
    }
    free(cs);
    free(sn);
}

/* The shifted block of frequency j (eq. precon2para: the j-th diagonal block
 * of I (x) A_0 + Lambda (x) A_1, generalised to s+1 blocks):
 *   hatA_j = alpha_j M + beta_j kappa K,  alpha_j = sum_m a_m w^{jm},
 *   beta_j = sum_m b_m w^{jm},  w = exp(-2 pi i/ell).
 * For C^T the symbol is conjugated (w -> 1/w). */
static void symbol(int scheme, int ell, double tau, int j, int transpose,
                   double complex *alpha, double complex *beta)
{
    double a[4], b[4];
    int mlo, mhi;
    or_toeplitz(scheme, tau, &mlo, &mhi, a, b);
    double complex al = 0.0, be = 0.0;
    for (int m = mlo; m <= mhi; ++m) {
        int p = (int)((((long long)j * m) % ell + ell) % ell);
        double ang = -2.0 * M_PI * p / ell;
        if (transpose) ang = -ang;
        double complex wp = cos(ang) + I * sin(ang);
        al += a[m - mlo] * wp;
        be += b[m - mlo] * wp;
    }
    *alpha = al;
    *beta = be;
}

void or_symbol(int scheme, int ell, double tau, int j, int transpose, double *out4)
{
    double complex al, be;
    symbol(scheme, ell, tau, j, transpose, &al, &be);
    out4[0] = creal(al); out4[1] = cimag(al);
    out4[2] = creal(be); out4[3] = cimag(be);
}

/* Complex Thomas (no pivoting) for hatA_j x = r: the paper's per-block solve
 * of Sec. 3.  Returns 0 or -4 on a zero pivot. */
static int thomas_cplx(int n, double complex d, double complex e,
                       const double complex *r, double complex *x, double complex *cp,
                       double complex *gp)
{
    double complex piv = d;
    if (piv == 0.0) return -4;
    cp[0] = e / piv;
    gp[0] = r[0] / piv;
    for (int i = 1; i < n; ++i) {
        piv = d - e * cp[i - 1];
        if (piv == 0.0) return -4;
        cp[i] = e / piv;
        gp[i] = (r[i] - e * gp[i - 1]) / piv;
    }
    x[n - 1] = gp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = gp[i] - cp[i] * x[i + 1];
    return 0;
}

/* Solve hatA_j Y_j = X_j for every frequency row j = 0..ell-1 of an ell x n
 * complex array (re/im planes), in place.  Every j is solved, the redundant
 * upper half of the spectrum included. */
int or_shifted_solve_all(int scheme, int n, int ell, double tau, double kappa, int transpose,
                         double *Xr, double *Xi)
{
    double h = 1.0 / (n + 1);
    int st = 0;
#pragma omp parallel
    {
        double complex *r = (double complex *)malloc(sizeof(double complex) * (size_t)n);
        double complex *x = (double complex *)malloc(sizeof(double complex) * (size_t)n);
        double complex *cp = (double complex *)malloc(sizeof(double complex) * (size_t)n);
        double complex *gp = (double complex *)malloc(sizeof(double complex) * (size_t)n);
#pragma omp for schedule(static)
        for (int j = 0; j < ell; ++j) {
            double complex al, be;
            symbol(scheme, ell, tau, j, transpose, &al, &be);
            double complex d = al * (4.0 * h / 6.0) + be * kappa * (2.0 / h);
            double complex e = al * (h / 6.0) - be * kappa * (1.0 / h);
            for (int i = 0; i < n; ++i) r[i] = Xr[(size_t)j * n + i] + I * Xi[(size_t)j * n + i];
            int s = thomas_cplx(n, d, e, r, x, cp, gp);
            if (s) {
#pragma omp atomic write
                st = s;
            }
            for (int i = 0; i < n; ++i) {
                Xr[(size_t)j * n + i] = creal(x[i]);
                Xi[(size_t)j * n + i] = cimag(x[i]);
            }
        }
        free(r); free(x); free(cp); free(gp);
    }
    return st;
}

/* z = C^{-1} r (or C^{-T} r) by the Fourier diagonalisation of eq. precon2para:
 * direct DFT along time, the shifted solves, inverse direct DFT.  The result of
 * the inverse transform is real up to rounding; the largest |Im| relative to the
 * largest |Re| is returned in *imag_ratio. */
int or_pinv_direct(int scheme, int n, int ell, double tau, double kappa, int transpose,
                   const double *r, double *z, double *imag_ratio)
{
    size_t N = (size_t)n * ell;
    double *Xr = (double *)malloc(sizeof(double) * N);
    double *Xi = (double *)malloc(sizeof(double) * N);
    double *Zi = (double *)malloc(sizeof(double) * N);
    or_dft(ell, n, r, NULL, Xr, Xi, 0);
    int st = or_shifted_solve_all(scheme, n, ell, tau, kappa, transpose, Xr, Xi);
    or_dft(ell, n, Xr, Xi, z, Zi, 1);
    double mr = 0.0, mi = 0.0;
    for (size_t p = 0; p < N; ++p) {
        if (fabs(z[p]) > mr) mr = fabs(z[p]);
        if (fabs(Zi[p]) > mi) mi = fabs(Zi[p]);
    }
    if (imag_ratio) *imag_ratio = (mr > 0.0) ? mi / mr : mi;
    free(Xr); free(Xi); free(Zi);
    return st;
}

/* --------------------------------------------------------------- gradient */

/* Reductions of the adjoint gradient for L(U) with A(kappa) U = b(u_0, v_0, kappa):
 *   dL/du_0 = (db/du_0)^T l,  dL/dv_0 = (db/dv_0)^T l,
 *   dL/dkappa = l^T db/dkappa - l^T (dA/dkappa) U,
 * with (dA/dkappa U)_k = sum_m (K coefficient of block (k, k-m)) K u_{k-m}.
 * heat: b_1 = M u_0 -> g_u0 = M l_1, no kappa term in b.
 * BD2:  b_1 = A_0 (u_0 + tau v_0), b_2 = -M u_0 ->
 *       g_u0 = A_0 l_1 - M l_2, g_v0 = tau A_0 l_1,
 *       db_1/dkappa = tau^2 K (u_0 + tau v_0).
 * BD4:  b_1 = B (u_0 + tau v_0), b_2 = -M u_0, b_3 = M u_0 (B = BD2's A_0) ->
 *       g_u0 = B l_1 - M l_2 + M l_3, g_v0 = tau B l_1, db_1/dkappa as BD2.
 * CD:   b_1 = -M u_0 -> g_u0 = -M l_1, g_v0 = 0, no kappa term in b. */
int or_grad(int scheme, int n, int ell, double tau, double kappa, const double *tau_k,
            const double *u0, const double *v0, const double *U, const double *L,
            double *g_u0, double *g_v0, double *g_kappa)
{
    double a[4], b[4];
    int mlo, mhi;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0) return -1;
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    double gk = 0.0;
    for (int k = 0; k < ell; ++k) {
        for (int m = mlo; m <= mhi; ++m) {
            double cm, bm;   /* with kappa = 1 the K coefficient is dA/dkappa's */
            if (!or_block(scheme, tau, 1.0, tau_k, ell, k, m, &cm, &bm) || bm == 0.0) continue;
            or_stiff_apply(n, U + (size_t)(k - m) * n, t);
            double dot = 0.0;
            for (int i = 0; i < n; ++i) dot += L[(size_t)k * n + i] * t[i];
            gk -= bm * dot;
        }
    }
    if (g_v0) memset(g_v0, 0, sizeof(double) * (size_t)n);
    if (scheme == OR_HEAT) {
        or_mass_apply(n, L, g_u0);
    } else if (scheme == OR_CD) {
        mk_apply(n, -1.0, 0.0, L, g_u0);
    } else {
        double *w = (double *)malloc(sizeof(double) * (size_t)n);
        mk_apply(n, 1.0, tau * tau * kappa, L, g_u0);
        or_mass_apply(n, L + n, t);
        for (int i = 0; i < n; ++i) g_u0[i] -= t[i];
        if (scheme == OR_BD4) {
            or_mass_apply(n, L + 2 * (size_t)n, t);
            for (int i = 0; i < n; ++i) g_u0[i] += t[i];
        }
        if (g_v0) {
            mk_apply(n, 1.0, tau * tau * kappa, L, g_v0);
            for (int i = 0; i < n; ++i) g_v0[i] *= tau;
        }
        for (int i = 0; i < n; ++i) w[i] = u0[i] + (v0 ? tau * v0[i] : 0.0);
        or_stiff_apply(n, w, t);
        double dot = 0.0;
        for (int i = 0; i < n; ++i) dot += L[i] * t[i];
        gk += tau * tau * dot;
        free(w);
    }
    *g_kappa = gk;
    free(t);
    return 0;
}
