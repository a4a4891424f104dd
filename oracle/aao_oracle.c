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
 *   - block m of the lower-triangular Toeplitz matrix is A_m = a_m M + b_m kappa K.
 *       heat, implicit Euler (eq. timestepproblem1, read as M + tau K):
 *             A_0 = M + tau kappa K, A_1 = -M
 *       wave, BD2 (eq. BD2 and the system C_BD2):
 *             A_0 = M + tau^2 kappa K, A_1 = -2M, A_2 = M
 *   - the DFT along time is X_j = sum_k x_k w^{jk}, w = exp(-2 pi i/ell).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_HEAT 0
#define OR_BD2 1

/* ---------------------------------------------------------------- scheme */

/* Block coefficients (a_m, b_m), m = 0..s, of the monolithic matrix.
 * Heat: eq. monolithicheat (A_0 = M + tau K after the implicit Euler step,
 * A_1 = -M).  Wave BD2: the system C_BD2 (A_0 = M + tau^2 K, A_1 = -2M,
 * A_2 = M).  Returns s, or -1 for an unknown scheme. */
int or_scheme_coeffs(int scheme, double tau, double *a, double *b)
{
    if (scheme == OR_HEAT) {
        a[0] = 1.0;  b[0] = tau;
        a[1] = -1.0; b[1] = 0.0;
        return 1;
    }
    if (scheme == OR_BD2) {
        a[0] = 1.0;  b[0] = tau * tau;
        a[1] = -2.0; b[1] = 0.0;
        a[2] = 1.0;  b[2] = 0.0;
        return 2;
    }
    return -1;
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
 * one or two are zero).
 *   heat (eq. monolithicheat): b_1 = M u_0.
 *   BD2  (system C_BD2): b_1 = A_0 (u_0 + tau v_0), b_2 = -M u_0; the first row
 *        is the start-up step u_1 = u_0 + tau v_0, which is the printed row
 *        A_0 u_1 = (M + tau^2 K) u_0 when the initial velocity v_0 is zero. */
int or_build_rhs(int scheme, int n, int ell, double tau, double kappa,
                 const double *u0, const double *v0, double *b)
{
    memset(b, 0, sizeof(double) * (size_t)n * (size_t)ell);
    if (scheme == OR_HEAT) {
        or_mass_apply(n, u0, b);
        return 0;
    }
    if (scheme == OR_BD2) {
        if (ell < 2) return -1;
        double *w = (double *)malloc(sizeof(double) * (size_t)n);
        for (int i = 0; i < n; ++i) w[i] = u0[i] + (v0 ? tau * v0[i] : 0.0);
        mk_apply(n, 1.0, tau * tau * kappa, w, b);
        mk_apply(n, -1.0, 0.0, u0, b + n);
        free(w);
        return 0;
    }
    return -1;
}

/* The diagonal block of time level k (0-based row).  With variable steps
 * (heat only, eq. nonuniformmonolithicheat) A_0^k = M + tau_k kappa K. */
static void diag_block(int scheme, double tau, double kappa, const double *tau_k, int k,
                       double *cm, double *ck)
{
    double a[4], b[4];
    or_scheme_coeffs(scheme, tau, a, b);
    *cm = a[0];
    *ck = b[0] * kappa;
    if (tau_k && scheme == OR_HEAT) *ck = tau_k[k] * kappa;
}

/* ------------------------------------------------------ monolithic matvec */

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), where A is the block
 * lower-triangular Toeplitz matrix of eq. monolithicheat / C_BD2, or the
 * variable-step matrix B of eq. nonuniformmonolithicheat when tau_k != NULL.
 * Row k: (A x)_k = sum_{m=0}^{min(s,k)} A_m x_{k-m}; every block is symmetric,
 * so (A^T x)_k = sum_{m=0}^{min(s, ell-1-k)} A_m^{(k+m)} x_{k+m}. */
int or_apply_A(int scheme, int n, int ell, double tau, double kappa, const double *tau_k,
               const double *x, double *y, int transpose)
{
    double a[4], b[4];
    int s = or_scheme_coeffs(scheme, tau, a, b);
    if (s < 0) return -1;
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    memset(y, 0, sizeof(double) * (size_t)n * (size_t)ell);
    for (int k = 0; k < ell; ++k) {
        for (int m = 0; m <= s; ++m) {
            int src = transpose ? k + m : k - m;
            if (src < 0 || src >= ell) continue;
            double cm = a[m], ck = b[m] * kappa;
            if (m == 0) diag_block(scheme, tau, kappa, tau_k, k, &cm, &ck);
            mk_apply(n, cm, ck, x + (size_t)src * n, t);
            for (int i = 0; i < n; ++i) y[(size_t)k * n + i] += t[i];
        }
    }
    free(t);
    return 0;
}

/* y = C x: the block circulant of eq. standardheatprecon / wavepreconditioner,
 * i.e. the same blocks wrapped around, (C x)_k = sum_m A_m x_{(k-m) mod ell}.
 * transpose = 1 gives C^T, (C^T x)_k = sum_m A_m x_{(k+m) mod ell}. */
int or_apply_C(int scheme, int n, int ell, double tau, double kappa,
               const double *x, double *y, int transpose)
{
    double a[4], b[4];
    int s = or_scheme_coeffs(scheme, tau, a, b);
    if (s < 0) return -1;
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    memset(y, 0, sizeof(double) * (size_t)n * (size_t)ell);
    for (int k = 0; k < ell; ++k) {
        for (int m = 0; m <= s; ++m) {
            int src = transpose ? (k + m) % ell : ((k - m) % ell + ell) % ell;
            mk_apply(n, a[m], b[m] * kappa, x + (size_t)src * n, t);
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

/* Forward block substitution: the exact solution of A U = b, i.e. the
 * sequential time stepping of eq. timestepproblem1 / BD2 that the monolithic
 * system packages:  u_k = A_0^{-1} (b_k - sum_{m=1}^{min(s,k)} A_m u_{k-m}). */
int or_solve_seq(int scheme, int n, int ell, double tau, double kappa, const double *tau_k,
                 const double *bvec, double *U)
{
    double a[4], b[4];
    int s = or_scheme_coeffs(scheme, tau, a, b);
    if (s < 0) return -1;
    double *rhs = (double *)malloc(sizeof(double) * (size_t)n);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    int st = 0;
    for (int k = 0; k < ell && st == 0; ++k) {
        memcpy(rhs, bvec + (size_t)k * n, sizeof(double) * (size_t)n);
        for (int m = 1; m <= s && m <= k; ++m) {
            mk_apply(n, a[m], b[m] * kappa, U + (size_t)(k - m) * n, t);
            for (int i = 0; i < n; ++i) rhs[i] -= t[i];
        }
        double cm, ck;
        diag_block(scheme, tau, kappa, tau_k, k, &cm, &ck);
        st = mk_solve(n, cm, ck, rhs, U + (size_t)k * n);
    }
    free(rhs);
    free(t);
    return st;
}

/* Backward block substitution: the exact solution of A^T L = g,
 * l_k = (A_0^k)^{-1} (g_k - sum_{m=1}^{min(s, ell-1-k)} A_m l_{k+m}). */
int or_adjoint_seq(int scheme, int n, int ell, double tau, double kappa, const double *tau_k,
                   const double *g, double *L)
{
    double a[4], b[4];
    int s = or_scheme_coeffs(scheme, tau, a, b);
    if (s < 0) return -1;
    double *rhs = (double *)malloc(sizeof(double) * (size_t)n);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    int st = 0;
    for (int k = ell - 1; k >= 0 && st == 0; --k) {
        memcpy(rhs, g + (size_t)k * n, sizeof(double) * (size_t)n);
        for (int m = 1; m <= s && k + m < ell; ++m) {
            mk_apply(n, a[m], b[m] * kappa, L + (size_t)(k + m) * n, t);
            for (int i = 0; i < n; ++i) rhs[i] -= t[i];
        }
        double cm, ck;
        diag_block(scheme, tau, kappa, tau_k, k, &cm, &ck);
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
    int s = or_scheme_coeffs(scheme, tau, a, b);
    double complex al = 0.0, be = 0.0;
    for (int m = 0; m <= s; ++m) {
        int p = (int)(((long long)j * m) % ell);
        double ang = -2.0 * M_PI * p / ell;
        if (transpose) ang = -ang;
        double complex wp = cos(ang) + I * sin(ang);
        al += a[m] * wp;
        be += b[m] * wp;
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
 * with (dA/dkappa U)_k = sum_m b_m^{(k)} K u_{k-m}.
 * heat: b_1 = M u_0 -> g_u0 = M l_1, no kappa term in b.
 * BD2:  b_1 = A_0 (u_0 + tau v_0), b_2 = -M u_0 ->
 *       g_u0 = A_0 l_1 - M l_2, g_v0 = tau A_0 l_1,
 *       db_1/dkappa = tau^2 K (u_0 + tau v_0). */
int or_grad(int scheme, int n, int ell, double tau, double kappa, const double *tau_k,
            const double *u0, const double *v0, const double *U, const double *L,
            double *g_u0, double *g_v0, double *g_kappa)
{
    double a[4], b[4];
    int s = or_scheme_coeffs(scheme, tau, a, b);
    if (s < 0) return -1;
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    double gk = 0.0;
    for (int k = 0; k < ell; ++k) {
        for (int m = 0; m <= s && m <= k; ++m) {
            double bm = b[m];
            if (m == 0 && tau_k && scheme == OR_HEAT) bm = tau_k[k];
            if (bm == 0.0) continue;
            or_stiff_apply(n, U + (size_t)(k - m) * n, t);
            double dot = 0.0;
            for (int i = 0; i < n; ++i) dot += L[(size_t)k * n + i] * t[i];
            gk -= bm * dot;
        }
    }
    if (scheme == OR_HEAT) {
        or_mass_apply(n, L, g_u0);
        if (g_v0) memset(g_v0, 0, sizeof(double) * (size_t)n);
    } else {
        double *w = (double *)malloc(sizeof(double) * (size_t)n);
        mk_apply(n, 1.0, tau * tau * kappa, L, g_u0);
        or_mass_apply(n, L + n, t);
        for (int i = 0; i < n; ++i) g_u0[i] -= t[i];
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
