"""Pins of the CPU oracle against mathematics that does not come from the oracle:
quadrature, closed forms in the discrete sine basis, dense Kronecker assembly
with LAPACK solves/eigenvalues, textbook DFT properties and finite differences.
Each test names the property and the passage of arXiv 1810.00615 it pins."""
import numpy as np
import pytest
from scipy import integrate

import pins

HEAT, BD2 = 0, 1


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# ---------------------------------------------------------------- Sec. 2 space

def test_mass_stiffness_match_quadrature(orc):
    """M, K of eq. applyEuler are the Galerkin integrals of the hat functions."""
    n = 7
    M, K = pins.quad_MK(n)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(n)
    assert rel(orc.mass(n, x), M @ x) < 1e-13
    assert rel(orc.stiff(n, x), K @ x) < 1e-13


def test_sine_modes_are_eigenvectors(orc):
    """Generalised eigenpairs of (K, M): lambda_m = 6(1-cos m pi h)/(h^2 (2+cos m pi h))."""
    n = 15
    for m in (1, 2, 7, 15):
        s = pins.sine_vec(n, m)
        assert rel(orc.mass(n, s), pins.mu(n, m) * s) < 1e-14
        assert rel(orc.stiff(n, s), pins.lam(n, m) * pins.mu(n, m) * s) < 1e-13
    M, K = pins.quad_MK(n)
    from scipy.linalg import eigh
    ev = eigh(K, M, eigvals_only=True)
    assert rel(np.sort(ev), pins.lam(n, np.arange(1, n + 1))) < 1e-13


def test_load_vector_matches_quadrature(orc):
    """The L2 load vector of a sine series (initial data of eq. timestepproblem1)."""
    n = 9
    modes = np.array([1, 3, 4], dtype=np.int32)
    amps = np.array([1.0, -0.3, 0.2])
    s = lambda x: sum(a * np.sin(q * np.pi * x) for q, a in zip(modes, amps))
    h = 1.0 / (n + 1)
    f = np.empty(n)
    for i in range(1, n + 1):
        phi, a, b = pins.hat(i, n)
        f[i - 1] = (integrate.quad(lambda x: s(x) * phi(x), a, i * h, epsabs=1e-15)[0]
                    + integrate.quad(lambda x: s(x) * phi(x), i * h, b, epsabs=1e-15)[0])
    assert rel(orc.load_sine(n, modes, amps), f) < 1e-12
    M, _ = pins.quad_MK(n)
    assert rel(orc.project_sine(n, modes, amps), np.linalg.solve(M, f)) < 1e-12


# ----------------------------------------------------- exact sequential solves

@pytest.mark.parametrize("kappa", [1.0, 1.7])
def test_heat_sequential_solve_closed_form(orc, kappa):
    """Implicit Euler (eq. timestepproblem1, read as M + tau K) has the discrete sine
    closed form u_k = sum_m c_m (1 + tau kappa lambda_m)^{-k} s_m."""
    n, ell = 31, 40
    tau = 1.0 / ell
    u0 = orc.project_sine(n, np.arange(1, 8, dtype=np.int32), np.linspace(1, -0.5, 7))
    b = orc.build_rhs(HEAT, n, ell, tau, kappa, u0)
    U = orc.solve_seq(HEAT, n, ell, tau, kappa, b)
    assert rel(U, pins.heat_closed_form(u0, ell, tau, kappa)) < 1e-13


def test_bd2_sequential_solve_closed_form(orc):
    """BD2 (system C_BD2) with initial velocity: per-mode damped oscillation."""
    n, ell = 23, 50
    tau = 1.0 / ell
    rng = np.random.default_rng(3)
    u0 = pins.sine_synth(np.r_[rng.standard_normal(6), np.zeros(n - 6)])
    v0 = pins.sine_synth(np.r_[rng.standard_normal(5), np.zeros(n - 5)])
    b = orc.build_rhs(BD2, n, ell, tau, 1.3, u0, v0)
    U = orc.solve_seq(BD2, n, ell, tau, 1.3, b)
    assert rel(U, pins.bd2_closed_form(u0, v0, ell, tau, 1.3)) < 1e-12


@pytest.mark.parametrize("scheme", [HEAT, BD2])
def test_monolithic_matches_dense_kronecker(orc, scheme):
    """apply_A / apply_A^T / apply_C / solve_seq / adjoint_seq against the assembled
    sum_m Shift^m (x) A_m (eq. monolithicheat, C_BD2, eq. standardheatprecon,
    eq. wavepreconditioner) with M, K from quadrature."""
    n, ell, tau, kappa = 5, 7, 0.13, 0.8
    M, K = pins.quad_MK(n)
    if scheme == HEAT:
        blocks = [M + tau * kappa * K, -M]
    else:
        blocks = [M + tau * tau * kappa * K, -2 * M, M]
    A = pins.kron_A(blocks, ell)
    C = pins.kron_A(blocks, ell, circulant=True)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(n * ell)
    assert rel(orc.apply_A(scheme, n, ell, tau, kappa, x), A @ x) < 1e-13
    assert rel(orc.apply_A(scheme, n, ell, tau, kappa, x, transpose=True), A.T @ x) < 1e-13
    assert rel(orc.apply_C(scheme, n, ell, tau, kappa, x), C @ x) < 1e-13
    assert rel(orc.apply_C(scheme, n, ell, tau, kappa, x, transpose=True), C.T @ x) < 1e-13
    assert rel(orc.solve_seq(scheme, n, ell, tau, kappa, x), np.linalg.solve(A, x)) < 1e-12
    assert rel(orc.adjoint_seq(scheme, n, ell, tau, kappa, x), np.linalg.solve(A.T, x)) < 1e-12


def test_variable_steps_and_E_split(orc):
    """Eq. nonuniformmonolithicheat and Q = P + sigma (x) K: B - A(tau) = blockdiag(sigma_k K)."""
    n, ell, kappa = 4, 6, 1.1
    tau = 1.0 / ell
    tk = tau * (1 + 0.3 * np.sin(np.arange(ell)))
    M, K = pins.quad_MK(n)
    B = pins.kron_A([M, -M], ell) + np.kron(np.diag(tk), kappa * K)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(n * ell)
    assert rel(orc.apply_A(HEAT, n, ell, tau, kappa, x, tau_k=tk), B @ x) < 1e-13
    assert rel(orc.apply_A(HEAT, n, ell, tau, kappa, x, transpose=True, tau_k=tk), B.T @ x) < 1e-13
    # Q of eq. nonunistandardheatprecon: B with -M wrapped into the corner
    Q = B + np.kron(np.eye(ell, k=ell - 1), -M)
    E = np.kron(np.diag(tk - tau), kappa * K)
    assert rel(orc.apply_E(n, ell, tau, kappa, tk, x), E @ x) < 1e-13
    assert rel(orc.apply_C(HEAT, n, ell, tau, kappa, x).ravel()
               + orc.apply_E(n, ell, tau, kappa, tk, x).ravel(), Q @ x) < 1e-13
    assert rel(orc.solve_seq(HEAT, n, ell, tau, kappa, x, tau_k=tk), np.linalg.solve(B, x)) < 1e-12


# ----------------------------------------------------------- Fourier, Sec. 3

def test_direct_dft_textbook_properties(orc):
    ell, n = 12, 3
    rng = np.random.default_rng(4)
    x = rng.standard_normal((ell, n)) + 1j * rng.standard_normal((ell, n))
    X = orc.dft(x)
    assert rel(X, np.fft.fft(x, axis=0)) < 1e-14              # library routine
    assert rel(orc.dft(X, inverse=True), x) < 1e-14            # inverse
    assert abs(np.sum(abs(X) ** 2) / ell - np.sum(abs(x) ** 2)) < 1e-12 * np.sum(abs(x) ** 2)
    const = orc.dft(np.ones((ell, 1)))
    assert abs(const[0, 0] - ell) < 1e-13 and np.max(abs(const[1:])) < 1e-13
    k0 = 5                                                       # single frequency -> delta
    wave = np.exp(-2j * np.pi * k0 * np.arange(ell) / ell)[:, None]
    D = orc.dft(wave, inverse=True)
    assert abs(D[(-k0) % ell, 0] - 1) < 1e-14 or abs(D[k0, 0] - 1) < 1e-14
    assert np.sum(abs(D) > 1e-12) == 1


@pytest.mark.parametrize("scheme", [HEAT, BD2])
def test_symbol_and_shifted_solves(orc, scheme):
    """hatA_j = alpha_j M + beta_j kappa K, the diagonal blocks of eq. precon2para:
    heat alpha_j = 1 - w^j, beta_j = tau; BD2 alpha_j = (1 - w^j)^2, beta_j = tau^2."""
    n, ell, tau, kappa = 6, 10, 0.1, 1.4
    M, K = pins.quad_MK(n)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((ell, n)) + 1j * rng.standard_normal((ell, n))
    for tr in (False, True):
        Y = orc.shifted_solve_all(scheme, n, ell, tau, kappa, X, transpose=tr)
        for j in range(ell):
            w = np.exp((1 if tr else -1) * 2j * np.pi * j / ell)
            al, be = (1 - w, tau) if scheme == HEAT else ((1 - w) ** 2, tau * tau)
            a2, b2 = orc.symbol(scheme, ell, tau, j, tr)
            assert abs(a2 - al) < 1e-14 and abs(b2 - be) < 1e-15
            Aj = al * M + be * kappa * K
            assert rel(Y[j], np.linalg.solve(Aj, X[j])) < 1e-12


@pytest.mark.parametrize("scheme", [HEAT, BD2])
@pytest.mark.parametrize("ell", [1, 2, 3, 8, 9])
def test_pinv_is_circulant_inverse(orc, scheme, ell):
    """C^{-1} r via eq. precon2para equals the dense solve with the block circulant,
    and C^{-1}(C x) = x; the result of the inverse transform is real."""
    n, kappa = 5, 0.9
    tau = 1.0 / max(ell, 1)
    M, K = pins.quad_MK(n)
    blocks = [M + tau * kappa * K, -M] if scheme == HEAT else \
        [M + tau * tau * kappa * K, -2 * M, M]
    C = np.zeros((n * ell, n * ell))      # blocks wrap mod ell, also when ell <= s
    for m, B in enumerate(blocks):
        for k in range(ell):
            src = (k - m) % ell
            C[k * n:(k + 1) * n, src * n:(src + 1) * n] += B
    rng = np.random.default_rng(6)
    r = rng.standard_normal(n * ell)
    for tr in (False, True):
        z, ratio = orc.pinv_direct(scheme, n, ell, tau, kappa, r, transpose=tr)
        ref = np.linalg.solve(C.T if tr else C, r)
        assert rel(z, ref) < 1e-11
        assert ratio < 1e-13
        assert rel(orc.pinv(scheme, n, ell, tau, kappa, r, transpose=tr), z) < 1e-12
        Cx = orc.apply_C(scheme, n, ell, tau, kappa, r, transpose=tr)
        assert rel(orc.pinv_direct(scheme, n, ell, tau, kappa, Cx, transpose=tr)[0], r) < 1e-11


def test_heat_preconditioned_spectrum(orc):
    """eig(C^{-1} A) = {1} (n ell - n times) and nu_m = 1/(1 - (1 + tau kappa lambda_m)^{-ell})."""
    n, ell, kappa = 5, 6, 1.0
    tau = 0.05 / ell
    N = n * ell
    I = np.eye(N)
    CinvA = np.column_stack([orc.pinv_direct(HEAT, n, ell, tau, kappa,
                                             orc.apply_A(HEAT, n, ell, tau, kappa, I[:, c]))[0].ravel()
                             for c in range(N)])
    ev = np.linalg.eigvals(CinvA)
    nu = 1.0 / (1.0 - (1.0 + tau * kappa * pins.lam(n, np.arange(1, n + 1))) ** (-ell))
    nonunit = ev[np.abs(ev - 1.0) > 1e-8]
    assert len(nonunit) == n
    assert np.max(np.abs(np.sort(nonunit.real) - np.sort(nu))) < 1e-10 * np.max(nu)
    assert np.max(np.abs(nonunit.imag)) < 1e-10


def test_bd2_preconditioned_rank(orc):
    """A - C is a corner of rank <= s n: C^{-1} A has exactly 2n non-unit eigenvalues for BD2."""
    n, ell, kappa = 4, 8, 1.0
    tau = 1.0 / ell
    N = n * ell
    I = np.eye(N)
    CinvA = np.column_stack([orc.pinv_direct(BD2, n, ell, tau, kappa,
                                             orc.apply_A(BD2, n, ell, tau, kappa, I[:, c]))[0].ravel()
                             for c in range(N)])
    ev = np.linalg.eigvals(CinvA)
    assert np.sum(np.abs(ev - 1.0) > 1e-8) == 2 * n


def test_neumann_series(orc):
    """Eq. preconapprox1: the recurrence equals the truncated series sum (-C^{-1}E)^m C^{-1};
    with uniform steps (sigma = 0) every order equals order 0."""
    n, ell, kappa = 4, 6, 1.0
    tau = 1.0 / ell
    tk = tau * (1 + 0.4 * np.cos(np.arange(ell) * 1.3))
    M, K = pins.quad_MK(n)
    C = pins.kron_A([M + tau * kappa * K, -M], ell, circulant=True)
    E = np.kron(np.diag(tk - tau), kappa * K)
    Ci = np.linalg.inv(C)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(n * ell)
    for q in range(3):
        series = sum(np.linalg.matrix_power(-Ci @ E, m) @ Ci @ r for m in range(q + 1))
        assert rel(orc.neumann(HEAT, n, ell, tau, kappa, tk, r, q, direct=True), series) < 1e-11
        assert rel(orc.neumann(HEAT, n, ell, tau, kappa, tk, r, q), series) < 1e-11
        z0 = orc.neumann(HEAT, n, ell, tau, kappa, np.full(ell, tau), r, q)
        assert rel(z0, Ci @ r) < 1e-12


# -------------------------------------------------------------------- GMRES

def test_fgmres_identity_preconditioner_dense(orc):
    """Textbook GMRES on a small non-symmetric system reaches the LAPACK solution."""
    rng = np.random.default_rng(8)
    A = np.eye(30) * 4 + rng.standard_normal((30, 30)) * 0.3
    b = rng.standard_normal(30)
    x, info = orc.fgmres(lambda v: A @ v, lambda v: v, b, restart=10, tol=1e-12, maxit=200)
    assert info["converged"] and info["true"] <= 1e-12
    assert rel(x, np.linalg.solve(A, b)) < 1e-10


@pytest.mark.parametrize("scheme,J", [(HEAT, 3), (BD2, 3)])
def test_fgmres_terminates_within_rank_bound(orc, scheme, J):
    """With C^{-1} (rank-s n correction) and data exciting J sine modes, GMRES terminates in
    at most s J + 1 iterations and returns the exact sequential solution."""
    n, ell, kappa = 15, 16, 1.0
    tau = 1.0 / ell
    rng = np.random.default_rng(9)
    u0 = pins.sine_synth(np.r_[rng.standard_normal(J), np.zeros(n - J)])
    v0 = pins.sine_synth(np.r_[rng.standard_normal(J), np.zeros(n - J)]) if scheme == BD2 else None
    b = orc.build_rhs(scheme, n, ell, tau, kappa, u0, v0).ravel()
    s = 1 if scheme == HEAT else 2
    x, info = orc.fgmres(lambda v: orc.apply_A(scheme, n, ell, tau, kappa, v).ravel(),
                         lambda v: orc.pinv(scheme, n, ell, tau, kappa, v).ravel(),
                         b, restart=50, tol=1e-13, maxit=100)
    assert info["converged"]
    assert info["iters"] <= s * J + 1
    U = orc.solve_seq(scheme, n, ell, tau, kappa, b)
    assert rel(x, U) < 1e-10


# ------------------------------------------------------------------ adjoint

def test_adjoint_gradient_fd_and_sine_basis(orc):
    """Gradient of L = 1/2 ||U - U_tgt||^2 w.r.t. u_0 and kappa via the transposed solve,
    against central finite differences on exact solves and, for u_0, against the
    scalar per-mode adjoint recursion in the sine basis."""
    n, ell = 9, 10
    tau = 1.0 / ell
    kappa = 1.25
    rng = np.random.default_rng(10)
    u0 = rng.standard_normal(n)
    U_t = orc.solve_seq(HEAT, n, ell, tau, 1.0, orc.build_rhs(HEAT, n, ell, tau, 1.0, rng.standard_normal(n)))

    def loss(u, k):
        U = orc.solve_seq(HEAT, n, ell, tau, k, orc.build_rhs(HEAT, n, ell, tau, k, u))
        return 0.5 * np.sum((U - U_t) ** 2), U
    L0, U = loss(u0, kappa)
    lam_ = orc.adjoint_seq(HEAT, n, ell, tau, kappa, U - U_t)
    gu, _, gk = orc.grad(HEAT, n, ell, tau, kappa, u0, U, lam_)
    hh = 1e-6
    fd_k = (loss(u0, kappa + hh)[0] - loss(u0, kappa - hh)[0]) / (2 * hh)
    assert abs(gk - fd_k) < 1e-7 * max(1.0, abs(fd_k))
    d = rng.standard_normal(n)
    fd_u = (loss(u0 + hh * d, kappa)[0] - loss(u0 - hh * d, kappa)[0]) / (2 * hh)
    assert abs(gu @ d - fd_u) < 1e-7 * max(1.0, abs(fd_u))
    # sine basis: per mode m, (A^T l)_k = mu (1 + tau kappa lam) l_k - mu l_{k+1};
    # with D = U - U_t = sum c_{m,k} s_m and ||s_m||^2 = (n+1)/2
    m = np.arange(1, n + 1)
    G = np.array([pins.sine_coeffs(row) for row in (U - U_t)]) * (n + 1) / 2.0   # s_m^T D_k
    mu_m, lm = pins.mu(n, m), pins.lam(n, m)
    # in coordinates l_k = sum_m y_{m,k} s_m: mu (1+t k lm)(n+1)/2 y_k - mu (n+1)/2 y_{k+1} = G_k
    y = np.zeros((ell + 1, n))
    for k in range(ell - 1, -1, -1):
        y[k] = (G[k] / ((n + 1) / 2.0) + mu_m * y[k + 1]) / (mu_m * (1 + tau * kappa * lm))
    gu_sine = pins.sine_synth(mu_m * y[0])
    assert rel(gu, gu_sine) < 1e-12


def test_bd2_adjoint_gradient_fd_and_sine_basis(orc):
    """BD2 gradients (system C_BD2 with the start-up row u_1 = u_0 + tau v_0):
    g_u0 = A_0 l_1 - M l_2, g_v0 = tau A_0 l_1 and
    g_kappa = l_1 . tau^2 K (u_0 + tau v_0) - tau^2 sum_k l_k . K u_k, against central
    finite differences on exact solves and, for g_u0 and g_v0, against the scalar
    per-mode adjoint recursion in the discrete sine basis."""
    n, ell = 11, 16
    tau = 1.0 / ell
    kappa = 1.3
    rng = np.random.default_rng(11)
    u0 = rng.standard_normal(n)
    v0 = rng.standard_normal(n)
    U_t = orc.solve_seq(BD2, n, ell, tau, 1.0,
                        orc.build_rhs(BD2, n, ell, tau, 1.0, rng.standard_normal(n),
                                      rng.standard_normal(n)))

    def loss(u, v, k):
        U = orc.solve_seq(BD2, n, ell, tau, k, orc.build_rhs(BD2, n, ell, tau, k, u, v))
        return 0.5 * np.sum((U - U_t) ** 2), U
    _, U = loss(u0, v0, kappa)
    lam_ = orc.adjoint_seq(BD2, n, ell, tau, kappa, U - U_t)
    gu, gv, gk = orc.grad(BD2, n, ell, tau, kappa, u0, U, lam_, v0=v0)
    hh = 1e-6
    fd_k = (loss(u0, v0, kappa + hh)[0] - loss(u0, v0, kappa - hh)[0]) / (2 * hh)
    assert abs(gk - fd_k) < 1e-7 * max(1.0, abs(fd_k))
    d = rng.standard_normal(n)
    fd_u = (loss(u0 + hh * d, v0, kappa)[0] - loss(u0 - hh * d, v0, kappa)[0]) / (2 * hh)
    assert abs(gu @ d - fd_u) < 1e-7 * max(1.0, abs(fd_u))
    fd_v = (loss(u0, v0 + hh * d, kappa)[0] - loss(u0, v0 - hh * d, kappa)[0]) / (2 * hh)
    assert abs(gv @ d - fd_v) < 1e-7 * max(1.0, abs(fd_v))
    # sine basis: on mode m the blocks act as mu (1 + tau^2 kappa lam), -2 mu, mu; with
    # l_k = sum_m y_{m,k} s_m and ||s_m||^2 = (n+1)/2 the adjoint rows read
    # mu (1 + tau^2 kappa lam) y_k - 2 mu y_{k+1} + mu y_{k+2} = G_k / ((n+1)/2)
    m = np.arange(1, n + 1)
    nrm = (n + 1) / 2.0
    G = np.array([pins.sine_coeffs(row) for row in (U - U_t)]) * nrm
    mu_m, lm = pins.mu(n, m), pins.lam(n, m)
    a0 = mu_m * (1 + tau * tau * kappa * lm)
    y = np.zeros((ell + 2, n))
    for k in range(ell - 1, -1, -1):
        y[k] = (G[k] / nrm + 2 * mu_m * y[k + 1] - mu_m * y[k + 2]) / a0
    assert rel(gu, pins.sine_synth(a0 * y[0] - mu_m * y[1])) < 1e-11
    assert rel(gv, pins.sine_synth(tau * a0 * y[0])) < 1e-11


def test_variable_step_gradient_fd(orc):
    """Heat with variable steps (eq. nonuniformmonolithicheat, A_0^k = M + tau_k kappa K):
    g_kappa = -sum_k tau_k l_k . K u_k and g_u0 = M l_1, against central finite
    differences on exact solves."""
    n, ell = 10, 12
    tau = 1.0 / ell
    tk = tau * (1 + 0.4 * np.sin(1.7 * np.arange(ell)))
    kappa = 0.9
    rng = np.random.default_rng(12)
    u0 = rng.standard_normal(n)
    U_t = rng.standard_normal((ell, n)) * 0.1

    def loss(u, k):
        U = orc.solve_seq(HEAT, n, ell, tau, k, orc.build_rhs(HEAT, n, ell, tau, k, u), tau_k=tk)
        return 0.5 * np.sum((U - U_t) ** 2), U
    _, U = loss(u0, kappa)
    lam_ = orc.adjoint_seq(HEAT, n, ell, tau, kappa, U - U_t, tau_k=tk)
    gu, gv, gk = orc.grad(HEAT, n, ell, tau, kappa, u0, U, lam_, tau_k=tk)
    hh = 1e-6
    fd_k = (loss(u0, kappa + hh)[0] - loss(u0, kappa - hh)[0]) / (2 * hh)
    assert abs(gk - fd_k) < 1e-7 * max(1.0, abs(fd_k))
    d = rng.standard_normal(n)
    fd_u = (loss(u0 + hh * d, kappa)[0] - loss(u0 - hh * d, kappa)[0]) / (2 * hh)
    assert abs(gu @ d - fd_u) < 1e-7 * max(1.0, abs(fd_u))
    assert np.all(gv == 0.0)


# ------------------------------------------------- BD4 and central differences

BD4, CD = 2, 3


def dense_scheme(scheme, n, ell, tau, kappa, circulant=False):
    """The printed monolithic matrices (and their circulants) assembled from M, K by
    quadrature: C_BD4 with its two start-up rows B, (C, B) and the Toeplitz rows
    A_2 A_1 A_0 (A_3 from the fourth row), R_BD4; C_CD with M beside the diagonal
    block tau^2 K - 2M, R_CD."""
    M, K = pins.quad_MK(n)
    N = n * ell
    A = np.zeros((N, N))

    def put(k, c, B):
        if circulant:
            c %= ell
        elif not 0 <= c < ell:
            return
        A[k * n:(k + 1) * n, c * n:(c + 1) * n] += B
    if scheme == BD4:
        A0, A1, A2, A3 = 2 * M + tau * tau * kappa * K, -5 * M, 4 * M, -M
        for k in range(ell):
            if k < 2 and not circulant:
                put(k, k, M + tau * tau * kappa * K)
                if k == 1:
                    put(k, 0, -2 * M)
                continue
            for m, B in enumerate((A0, A1, A2, A3)):
                put(k, k - m, B)
    else:
        for k in range(ell):
            put(k, k - 1, M)
            put(k, k, tau * tau * kappa * K - 2 * M)
            put(k, k + 1, M)
    return A


@pytest.mark.parametrize("scheme", [BD4, CD])
def test_bd4_cd_match_dense_assembly(orc, scheme):
    """apply_A / A^T / C / C^T, the exact solves and the transposed solves of the BD4
    and central-difference systems against the printed block matrices."""
    n, ell, tau, kappa = 5, 9, 0.11, 0.8
    A = dense_scheme(scheme, n, ell, tau, kappa)
    C = dense_scheme(scheme, n, ell, tau, kappa, circulant=True)
    rng = np.random.default_rng(40 + scheme)
    x = rng.standard_normal(n * ell)
    assert rel(orc.apply_A(scheme, n, ell, tau, kappa, x), A @ x) < 1e-13
    assert rel(orc.apply_A(scheme, n, ell, tau, kappa, x, transpose=True), A.T @ x) < 1e-13
    assert rel(orc.apply_C(scheme, n, ell, tau, kappa, x), C @ x) < 1e-13
    assert rel(orc.apply_C(scheme, n, ell, tau, kappa, x, transpose=True), C.T @ x) < 1e-13
    assert rel(orc.solve_seq(scheme, n, ell, tau, kappa, x), np.linalg.solve(A, x)) < 1e-11
    assert rel(orc.adjoint_seq(scheme, n, ell, tau, kappa, x), np.linalg.solve(A.T, x)) < 1e-11


def test_bd4_sequential_solve_mode_recursion(orc):
    """C_BD4 with initial velocity against the per-mode scalar BD4 recursion."""
    n, ell = 23, 50
    tau = 1.0 / ell
    rng = np.random.default_rng(41)
    u0 = pins.sine_synth(np.r_[rng.standard_normal(6), np.zeros(n - 6)])
    v0 = pins.sine_synth(np.r_[rng.standard_normal(5), np.zeros(n - 5)])
    b = orc.build_rhs(BD4, n, ell, tau, 1.3, u0, v0)
    U = orc.solve_seq(BD4, n, ell, tau, 1.3, b)
    assert rel(U, pins.bd4_mode_recursion(u0, v0, ell, tau, 1.3)) < 1e-11


@pytest.mark.parametrize("n,ell", [(15, 40), (63, 64)])
def test_cd_solve_mode_form(orc, n, ell):
    """C_CD against its per-mode ell x ell tridiagonal systems in time (the indefinite
    diagonal blocks make elimination without pivoting across time levels unstable at
    the larger size; the oracle's banded solve pivots)."""
    tau = 1.0 / ell
    rng = np.random.default_rng(42)
    u0 = pins.sine_synth(np.r_[rng.standard_normal(5), np.zeros(n - 5)])
    b = orc.build_rhs(CD, n, ell, tau, 0.9, u0)
    U = orc.solve_seq(CD, n, ell, tau, 0.9, b)
    assert rel(U, pins.cd_mode_solve(u0, ell, tau, 0.9)) < 1e-10
    with pytest.raises(RuntimeError):                  # no initial velocity for C_CD
        orc.build_rhs(CD, n, ell, tau, 0.9, u0, u0)


@pytest.mark.parametrize("scheme", [BD4, CD])
def test_bd4_cd_symbol_and_pinv(orc, scheme):
    """Circulant symbols in closed form (BD4: alpha_j = (1 - w^j)^2 (2 - w^j); CD:
    alpha_j = -4 sin^2(pi j / ell), real), the shifted solves against dense solves, and
    C^{-1} against the dense circulant."""
    n, ell, tau, kappa = 6, 10, 0.1, 1.4
    M, K = pins.quad_MK(n)
    rng = np.random.default_rng(43)
    X = rng.standard_normal((ell, n)) + 1j * rng.standard_normal((ell, n))
    for tr in (False, True):
        Y = orc.shifted_solve_all(scheme, n, ell, tau, kappa, X, transpose=tr)
        for j in range(ell):
            w = np.exp((1 if tr else -1) * 2j * np.pi * j / ell)
            al = (1 - w) ** 2 * (2 - w) if scheme == BD4 else -4 * np.sin(np.pi * j / ell) ** 2
            a2, b2 = orc.symbol(scheme, ell, tau, j, tr)
            assert abs(a2 - al) < 1e-13 and abs(b2 - tau * tau) < 1e-15
            assert rel(Y[j], np.linalg.solve(al * M + tau * tau * kappa * K, X[j])) < 1e-11
    C = dense_scheme(scheme, n, ell, tau, kappa, circulant=True)
    r = rng.standard_normal(n * ell)
    for tr in (False, True):
        z, ratio = orc.pinv_direct(scheme, n, ell, tau, kappa, r, transpose=tr)
        assert rel(z, np.linalg.solve(C.T if tr else C, r)) < 1e-10 and ratio < 1e-12
        assert rel(orc.pinv(scheme, n, ell, tau, kappa, r, transpose=tr), z) < 1e-11


@pytest.mark.parametrize("scheme,bound", [(BD4, 3), (CD, 2)])
def test_bd4_cd_preconditioned_rank(orc, scheme, bound):
    """A - C is confined to the first rows (BD4: three rows, the start-up rows and the
    wrapped blocks) or to the two corner blocks (CD), so C^{-1} A has at most 3n / 2n
    eigenvalues other than 1 (exactly that many here)."""
    n, ell, kappa = 4, 10, 1.0
    tau = 1.0 / ell
    N = n * ell
    I = np.eye(N)
    CinvA = np.column_stack([orc.pinv_direct(scheme, n, ell, tau, kappa,
                                             orc.apply_A(scheme, n, ell, tau, kappa, I[:, c]))[0].ravel()
                             for c in range(N)])
    ev = np.linalg.eigvals(CinvA)
    assert np.sum(np.abs(ev - 1.0) > 1e-7) == bound * n


@pytest.mark.parametrize("scheme", [BD4, CD])
def test_bd4_cd_adjoint_gradient_fd(orc, scheme):
    """Gradients of L = 1/2 ||U - U_t||^2 for C_BD4 (g_u0 = B l_1 - M l_2 + M l_3,
    g_v0 = tau B l_1, g_kappa with the start-up row's tau^2 K (u_0 + tau v_0)) and C_CD
    (g_u0 = -M l_1) against central finite differences on exact solves."""
    n, ell = 9, 14
    tau = 1.0 / ell
    kappa = 1.2
    rng = np.random.default_rng(44 + scheme)
    u0 = rng.standard_normal(n)
    v0 = rng.standard_normal(n) if scheme == BD4 else None
    U_t = rng.standard_normal((ell, n)) * 0.1

    def loss(u, v, k):
        U = orc.solve_seq(scheme, n, ell, tau, k, orc.build_rhs(scheme, n, ell, tau, k, u, v))
        return 0.5 * np.sum((U - U_t) ** 2), U
    _, U = loss(u0, v0, kappa)
    lam_ = orc.adjoint_seq(scheme, n, ell, tau, kappa, U - U_t)
    gu, gv, gk = orc.grad(scheme, n, ell, tau, kappa, u0, U, lam_, v0=v0)
    hh = 1e-6
    fd_k = (loss(u0, v0, kappa + hh)[0] - loss(u0, v0, kappa - hh)[0]) / (2 * hh)
    assert abs(gk - fd_k) < 1e-7 * max(1.0, abs(fd_k))
    d = rng.standard_normal(n)
    fd_u = (loss(u0 + hh * d, v0, kappa)[0] - loss(u0 - hh * d, v0, kappa)[0]) / (2 * hh)
    assert abs(gu @ d - fd_u) < 1e-7 * max(1.0, abs(fd_u))
    if scheme == BD4:
        fd_v = (loss(u0, v0 + hh * d, kappa)[0] - loss(u0, v0 - hh * d, kappa)[0]) / (2 * hh)
        assert abs(gv @ d - fd_v) < 1e-7 * max(1.0, abs(fd_v))
    else:
        assert np.all(gv == 0.0)
