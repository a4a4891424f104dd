/*
 * Reference oracle, two space dimensions: the all-at-once systems of the 1D oracle
 * (aao_oracle.c) with the spatial operators of the unit square.  The paper works in
 * one space dimension throughout; Sec. 3 (Parallel Implementation) and Sec. 5
 * (Conclusions) note that with more than one dimension the spatial blocks stop being
 * tridiagonal and need another solver for the shifted systems.  The time structure,
 * the circulant and its Fourier diagonalisation are unchanged.
 *
 * TEST INFRASTRUCTURE ONLY, like aao_oracle.c: the plain CPU statement of what the GPU
 * library computes; shares no code with it.
 *
 * Space: bilinear (Q1) elements on a uniform grid of nx x ny interior nodes of
 * [0,1]^2, hx = 1/(nx+1), hy = 1/(ny+1), zero Dirichlet data.  The Q1 mass and
 * stiffness matrices are the tensor products of the 1D P1 ones,
 *     M2 = My (x) Mx,   K2 = Ky (x) Mx + My (x) Kx,
 * with M = (h/6) tridiag(1,4,1), K = (1/h) tridiag(-1,2,-1) in each direction.  A
 * vector of one time level is ny x nx, x fastest (node (ix, iy) at iy nx + ix).
 * The time structure (blocks a_m M2 + b_m kappa K2, start-up rows, circulant wrap)
 * is that of the 1D oracle (or_block, or_toeplitz, or_symbol).
 * Exact solves of the 2D blocks (symmetric positive definite for the time-stepping
 * blocks, complex symmetric with positive-definite real part for the heat symbol)
 * use Gaussian elimination on the band (half-bandwidth nx + 1) without pivoting.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

int or_block(int scheme, double tau, double kappa, const double *tau_k, int ell, int k, int m,
             double *cm, double *ck);
int or_toeplitz(int scheme, double tau, int *mlo, int *mhi, double *a, double *b);
void or_symbol(int scheme, int ell, double tau, int j, int transpose, double *out4);
void or_dft(int ell, int n, const double *xr, const double *xi, double *Xr, double *Xi,
            int inverse);

/* y = (cm M2 + ck K2) x for one time level:
 * M2 x = My (Mx x), K2 x = Ky (Mx x) + My (Kx x), Mx, Kx along x, My, Ky along y. */
void or2_mk_apply(int nx, int ny, double cm, double ck, const double *x, double *y)
{
    const double hx = 1.0 / (nx + 1), hy = 1.0 / (ny + 1);
    const size_t N = (size_t)nx * ny;
    double *mxx = (double *)malloc(sizeof(double) * N);   /* Mx along every row */
    double *kxx = (double *)malloc(sizeof(double) * N);   /* Kx along every row */
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
            const double *r = x + (size_t)iy * nx;
            const double l = ix > 0 ? r[ix - 1] : 0.0, c = r[ix], rr = ix < nx - 1 ? r[ix + 1] : 0.0;
            mxx[(size_t)iy * nx + ix] = (hx / 6.0) * (l + 4.0 * c + rr);
            kxx[(size_t)iy * nx + ix] = (1.0 / hx) * (-l + 2.0 * c - rr);
        }
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
            const size_t e = (size_t)iy * nx + ix;
            const double md = mxx[e], mu = iy > 0 ? mxx[e - nx] : 0.0, mo = iy < ny - 1 ? mxx[e + nx] : 0.0;
            const double kd = kxx[e], ku = iy > 0 ? kxx[e - nx] : 0.0, ko = iy < ny - 1 ? kxx[e + nx] : 0.0;
            const double My_m = (hy / 6.0) * (mu + 4.0 * md + mo);   /* My (Mx x) */
            const double Ky_m = (1.0 / hy) * (-mu + 2.0 * md - mo);  /* Ky (Mx x) */
            const double My_k = (hy / 6.0) * (ku + 4.0 * kd + ko);   /* My (Kx x) */
            y[e] = cm * My_m + ck * (Ky_m + My_k);
        }
    free(mxx);
    free(kxx);
}

/* The matrix cm M2 + ck K2 (complex coefficients) in band storage
 * band[e][f - e + bw], |f - e| <= bw = nx + 1. */
static void band_assemble(int nx, int ny, double complex cm, double complex ck,
                          double complex *band)
{
    const double hx = 1.0 / (nx + 1), hy = 1.0 / (ny + 1);
    const int bw = nx + 1, W = 2 * bw + 1;
    const size_t N = (size_t)nx * ny;
    memset(band, 0, sizeof(double complex) * N * W);
    /* 1D entries: M: diag 4h/6, off h/6; K: diag 2/h, off -1/h */
    const double mxd = 4.0 * hx / 6.0, mxo = hx / 6.0, kxd = 2.0 / hx, kxo = -1.0 / hx;
    const double myd = 4.0 * hy / 6.0, myo = hy / 6.0, kyd = 2.0 / hy, kyo = -1.0 / hy;
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
            const size_t e = (size_t)iy * nx + ix;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int jy = iy + dy, jx = ix + dx;
                    if (jy < 0 || jy >= ny || jx < 0 || jx >= nx) continue;
                    const double Mx = dx == 0 ? mxd : mxo, Kx = dx == 0 ? kxd : kxo;
                    const double My = dy == 0 ? myd : myo, Ky = dy == 0 ? kyd : kyo;
                    const double complex v = cm * (My * Mx) + ck * (Ky * Mx + My * Kx);
                    const long f = (long)jy * nx + jx;
                    band[e * W + (size_t)(f - (long)e + bw)] += v;
                }
        }
}

/* In-place band LU without pivoting (unit lower factor); -4 on a zero pivot. */
static int band_lu(size_t N, int bw, double complex *band)
{
    const int W = 2 * bw + 1;
    for (size_t k = 0; k < N; ++k) {
        const double complex piv = band[k * W + bw];
        if (piv == 0.0) return -4;
        const size_t iend = k + bw < N - 1 ? k + bw : N - 1;
        for (size_t i = k + 1; i <= iend; ++i) {
            double complex *ri = band + i * W;
            const double complex l = ri[k - i + bw] / piv;
            ri[k - i + bw] = l;
            if (l == 0.0) continue;
            const double complex *rk = band + k * W;
            for (size_t j = k + 1; j <= iend; ++j) ri[j - i + bw] -= l * rk[j - k + bw];
        }
    }
    return 0;
}

/* x = A^{-1} x with the factors of band_lu */
static void band_solve(size_t N, int bw, const double complex *band, double complex *x)
{
    const int W = 2 * bw + 1;
    for (size_t i = 0; i < N; ++i) {
        const size_t j0 = i > (size_t)bw ? i - bw : 0;
        for (size_t j = j0; j < i; ++j) x[i] -= band[i * W + (j - i + bw)] * x[j];
    }
    for (size_t ii = N; ii-- > 0;) {
        const size_t jend = ii + bw < N - 1 ? ii + bw : N - 1;
        for (size_t j = ii + 1; j <= jend; ++j) x[ii] -= band[ii * W + (j - ii + bw)] * x[j];
        x[ii] /= band[ii * W + bw];
    }
}

/* Solve (cm M2 + ck K2) u = r (real). */
int or2_mk_solve(int nx, int ny, double cm, double ck, const double *r, double *u)
{
    const size_t N = (size_t)nx * ny;
    const int bw = nx + 1;
    double complex *band = (double complex *)malloc(sizeof(double complex) * N * (2 * bw + 1));
    double complex *x = (double complex *)malloc(sizeof(double complex) * N);
    band_assemble(nx, ny, cm, ck, band);
    int st = band_lu(N, bw, band);
    if (st == 0) {
        for (size_t e = 0; e < N; ++e) x[e] = r[e];
        band_solve(N, bw, band, x);
        for (size_t e = 0; e < N; ++e) u[e] = creal(x[e]);
    }
    free(band);
    free(x);
    return st;
}

/* y = A x or A^T x of the monolithic 2D system (blocks of or_block with M2, K2). */
int or2_apply_A(int scheme, int nx, int ny, int ell, double tau, double kappa, const double *x,
                double *y, int transpose)
{
    double a[4], b[4];
    int mlo, mhi;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0) return -1;
    const size_t n = (size_t)nx * ny;
    double *t = (double *)malloc(sizeof(double) * n);
    memset(y, 0, sizeof(double) * n * (size_t)ell);
    for (int k = 0; k < ell; ++k)
        for (int m = mlo; m <= mhi; ++m) {
            double cm, ck;
            const int src = transpose ? k + m : k - m;
            const int row = transpose ? k + m : k;
            if (!or_block(scheme, tau, kappa, NULL, ell, row, m, &cm, &ck)) continue;
            or2_mk_apply(nx, ny, cm, ck, x + (size_t)src * n, t);
            for (size_t e = 0; e < n; ++e) y[(size_t)k * n + e] += t[e];
        }
    free(t);
    return 0;
}

/* y = C x (C^T x): the circulant of the Toeplitz blocks, wrapped mod ell. */
int or2_apply_C(int scheme, int nx, int ny, int ell, double tau, double kappa, const double *x,
                double *y, int transpose)
{
    double a[4], b[4];
    int mlo, mhi;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0) return -1;
    const size_t n = (size_t)nx * ny;
    double *t = (double *)malloc(sizeof(double) * n);
    memset(y, 0, sizeof(double) * n * (size_t)ell);
    for (int k = 0; k < ell; ++k)
        for (int m = mlo; m <= mhi; ++m) {
            int src = transpose ? k + m : k - m;
            src = ((src % ell) + ell) % ell;
            or2_mk_apply(nx, ny, a[m - mlo], b[m - mlo] * kappa, x + (size_t)src * n, t);
            for (size_t e = 0; e < n; ++e) y[(size_t)k * n + e] += t[e];
        }
    free(t);
    return 0;
}

/* Exact solve of the lower-triangular 2D systems by forward (transpose: backward)
 * block substitution; -1 for the two-sided central-difference scheme. */
int or2_solve_seq(int scheme, int nx, int ny, int ell, double tau, double kappa,
                  const double *bvec, double *U, int transpose)
{
    double a[4], b[4];
    int mlo, mhi;
    if (or_toeplitz(scheme, tau, &mlo, &mhi, a, b) != 0 || mlo < 0) return -1;
    const size_t n = (size_t)nx * ny;
    double *rhs = (double *)malloc(sizeof(double) * n);
    double *t = (double *)malloc(sizeof(double) * n);
    int st = 0;
    for (int kk = 0; kk < ell && st == 0; ++kk) {
        const int k = transpose ? ell - 1 - kk : kk;
        memcpy(rhs, bvec + (size_t)k * n, sizeof(double) * n);
        double cm, ck;
        for (int m = 1; m <= mhi; ++m) {
            const int src = transpose ? k + m : k - m;
            const int row = transpose ? k + m : k;
            if (!or_block(scheme, tau, kappa, NULL, ell, row, m, &cm, &ck)) continue;
            or2_mk_apply(nx, ny, cm, ck, U + (size_t)src * n, t);
            for (size_t e = 0; e < n; ++e) rhs[e] -= t[e];
        }
        or_block(scheme, tau, kappa, NULL, ell, k, 0, &cm, &ck);
        st = or2_mk_solve(nx, ny, cm, ck, rhs, U + (size_t)k * n);
    }
    free(rhs);
    free(t);
    return st;
}

/* Right-hand side of the 2D system: the rows of the 1D oracle's or_build_rhs with M2, K2
 *   heat b_1 = M2 u0;  BD2 b_1 = (M2 + tau^2 kappa K2)(u0 + tau v0), b_2 = -M2 u0;
 *   BD4 as BD2 plus b_3 = M2 u0;  CD b_1 = -M2 u0 (no v0).  -1 for a short ell. */
int or2_build_rhs(int scheme, int nx, int ny, int ell, double tau, double kappa,
                  const double *u0, const double *v0, double *bvec)
{
    const size_t n = (size_t)nx * ny;
    memset(bvec, 0, sizeof(double) * n * (size_t)ell);
    if (scheme == 0) {
        or2_mk_apply(nx, ny, 1.0, 0.0, u0, bvec);
        return 0;
    }
    if (scheme == 1 || scheme == 2) {
        /* BD2 (system C_BD2) and BD4 (eq. BD4, system C_BD4): the first row's block
         * (M2 + tau^2 kappa K2, BD4's start-up block B) acts on u_1 = u0 + tau v0;
         * the u0 terms of the following rows move to the right */
        if (ell < (scheme == 1 ? 2 : 3)) return -1;
        double *w = (double *)malloc(sizeof(double) * n);
        for (size_t e = 0; e < n; ++e) w[e] = u0[e] + (v0 ? tau * v0[e] : 0.0);
        or2_mk_apply(nx, ny, 1.0, tau * tau * kappa, w, bvec);
        or2_mk_apply(nx, ny, -1.0, 0.0, u0, bvec + n);
        if (scheme == 2) or2_mk_apply(nx, ny, 1.0, 0.0, u0, bvec + 2 * n);
        free(w);
        return 0;
    }
    if (scheme == 3) {
        /* central differences (eq. CenDiffDisc): M2 u_0 of the first row moves to the
         * right; no initial velocity enters */
        if (v0) return -1;
        or2_mk_apply(nx, ny, -1.0, 0.0, u0, bvec);
        return 0;
    }
    return -1;
}

/* z = C^{-1} r (C^{-T} r) by the Fourier diagonalisation in time (eq. precon2para): direct
 * DFT along time, for every frequency j the 2D complex solve
 * (alpha_j M2 + beta_j kappa K2) Y_j = X_j on the band, inverse DFT.  The largest |Im| of
 * the result relative to the largest |Re| goes to *imag_ratio. */
int or2_pinv_direct(int scheme, int nx, int ny, int ell, double tau, double kappa, int transpose,
                    const double *r, double *z, double *imag_ratio)
{
    const size_t n = (size_t)nx * ny, N = n * (size_t)ell;
    const int bw = nx + 1;
    double *Xr = (double *)malloc(sizeof(double) * N);
    double *Xi = (double *)malloc(sizeof(double) * N);
    double *Zi = (double *)malloc(sizeof(double) * N);
    double complex *band = (double complex *)malloc(sizeof(double complex) * n * (2 * bw + 1));
    double complex *x = (double complex *)malloc(sizeof(double complex) * n);
    or_dft(ell, (int)n, r, NULL, Xr, Xi, 0);
    int st = 0;
    for (int j = 0; j < ell && st == 0; ++j) {
        double s4[4];
        or_symbol(scheme, ell, tau, j, transpose, s4);
        const double complex al = s4[0] + I * s4[1], be = s4[2] + I * s4[3];
        band_assemble(nx, ny, al, be * kappa, band);
        st = band_lu(n, bw, band);
        if (st) break;
        for (size_t e = 0; e < n; ++e) x[e] = Xr[(size_t)j * n + e] + I * Xi[(size_t)j * n + e];
        band_solve(n, bw, band, x);
        for (size_t e = 0; e < n; ++e) {
            Xr[(size_t)j * n + e] = creal(x[e]);
            Xi[(size_t)j * n + e] = cimag(x[e]);
        }
    }
    if (st == 0) or_dft(ell, (int)n, Xr, Xi, z, Zi, 1);
    double mr = 0.0, mi = 0.0;
    for (size_t p = 0; st == 0 && p < N; ++p) {
        if (fabs(z[p]) > mr) mr = fabs(z[p]);
        if (fabs(Zi[p]) > mi) mi = fabs(Zi[p]);
    }
    if (imag_ratio) *imag_ratio = mr > 0.0 ? mi / mr : mi;
    free(Xr); free(Xi); free(Zi); free(band); free(x);
    return st;
}
