"""Pins of the two-dimensional oracle (Q1 elements on the unit square, the monolithic
time structure of Sec. 2): the Q1 mass and stiffness integrals by 2D quadrature, the
tensor-product assembly, the discrete-sine closed form of 2D implicit Euler, the
printed block structure assembled densely, the Fourier diagonalisation of the
circulant (eq. precon2para) against dense solves, and the structure of C^{-1} A - I."""
import numpy as np
import pytest
from scipy import integrate

import pins

HEAT, BD2 = 0, 1


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def dense_MK2(nx, ny):
    Mx, Kx = pins.quad_MK(nx)
    My, Ky = pins.quad_MK(ny)
    return np.kron(My, Mx), np.kron(Ky, Mx) + np.kron(My, Kx)


def test_q1_integrals_by_2d_quadrature():
    """Entries of M2 and K2 are the integrals of products of bilinear hat functions and of
    their gradients (2D quadrature), which the tensor products reproduce."""
    nx, ny = 3, 2
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    M2, K2 = dense_MK2(nx, ny)

    def phi(i, h):
        c = (i + 1) * h
        return (lambda t: max(0.0, 1.0 - abs(t - c) / h),
                lambda t: (1.0 / h if t < c else -1.0 / h) if abs(t - c) < h else 0.0)
    for (a, b) in [(0, 0), (0, 1), (1, 4), (2, 5), (0, 4)]:
        ax, ay = a % nx, a // nx
        bx, by = b % nx, b // nx
        pa, da = phi(ax, hx)
        pb, db = phi(bx, hx)
        qa, ea = phi(ay, hy)
        qb, eb = phi(by, hy)
        brk_x = [k * hx for k in range(nx + 2)]
        brk_y = [k * hy for k in range(ny + 2)]

        def quad2(f):
            tot = 0.0
            for x0, x1 in zip(brk_x[:-1], brk_x[1:]):
                for y0, y1 in zip(brk_y[:-1], brk_y[1:]):
                    tot += integrate.dblquad(lambda y, x: f(x, y), x0, x1, y0, y1,
                                             epsabs=1e-14, epsrel=1e-12)[0]
            return tot
        m = quad2(lambda x, y: pa(x) * qa(y) * pb(x) * qb(y))
        k = quad2(lambda x, y: da(x) * qa(y) * db(x) * qb(y) + pa(x) * ea(y) * pb(x) * eb(y))
        assert abs(M2[a, b] - m) < 1e-12 and abs(K2[a, b] - k) < 1e-10


def test_mk2_matches_tensor_assembly(orc):
    nx, ny = 5, 4
    M2, K2 = dense_MK2(nx, ny)
    x = np.random.default_rng(60).standard_normal(nx * ny)
    assert rel(orc.mk2(nx, ny, 1.3, -0.4, x), (1.3 * M2 - 0.4 * K2) @ x) < 1e-13
    assert rel(orc.mk2_solve(nx, ny, 1.0, 0.7, x), np.linalg.solve(M2 + 0.7 * K2, x)) < 1e-12


def test_heat2d_closed_form(orc):
    """2D implicit Euler: the sine products s_p (x) s_q are eigenvectors of (K2, M2) with
    lambda_pq = lambda^x_p + lambda^y_q, so u_k = sum c_pq (1 + tau kappa lambda_pq)^{-k}."""
    nx, ny, ell, kappa = 9, 7, 12, 0.8
    tau = 1.0 / ell
    rng = np.random.default_rng(61)
    C = np.zeros((ny, nx))
    C[:3, :4] = rng.standard_normal((3, 4))
    Sx = np.sin(np.pi * np.outer(np.arange(1, nx + 1), np.arange(1, nx + 1)) / (nx + 1))
    Sy = np.sin(np.pi * np.outer(np.arange(1, ny + 1), np.arange(1, ny + 1)) / (ny + 1))
    u0 = Sy.T @ C @ Sx                                    # sum_pq C[q, p] s_q(y) s_p(x)
    b = orc.build_rhs2(HEAT, nx, ny, ell, tau, kappa, u0)
    U = orc.solve_seq2(HEAT, nx, ny, ell, tau, kappa, b)
    lam = pins.lam(ny, np.arange(1, ny + 1))[:, None] + pins.lam(nx, np.arange(1, nx + 1))[None, :]
    for k in range(ell):
        ref = Sy.T @ (C * (1.0 + tau * kappa * lam) ** (-(k + 1))) @ Sx
        assert rel(U[k], ref.ravel()) < 1e-12


@pytest.mark.parametrize("scheme", [HEAT, BD2])
def test_2d_monolithic_matches_dense(orc, scheme):
    nx, ny, ell, tau, kappa = 3, 2, 5, 0.13, 0.9
    M2, K2 = dense_MK2(nx, ny)
    blocks = [M2 + tau * kappa * K2, -M2] if scheme == HEAT else \
        [M2 + tau * tau * kappa * K2, -2 * M2, M2]
    A = pins.kron_A(blocks, ell)
    C = pins.kron_A(blocks, ell, circulant=True)
    x = np.random.default_rng(62).standard_normal(nx * ny * ell)
    assert rel(orc.apply_A2(scheme, nx, ny, ell, tau, kappa, x), A @ x) < 1e-13
    assert rel(orc.apply_A2(scheme, nx, ny, ell, tau, kappa, x, transpose=True), A.T @ x) < 1e-13
    assert rel(orc.apply_C2(scheme, nx, ny, ell, tau, kappa, x), C @ x) < 1e-13
    assert rel(orc.apply_C2(scheme, nx, ny, ell, tau, kappa, x, transpose=True), C.T @ x) < 1e-13
    assert rel(orc.solve_seq2(scheme, nx, ny, ell, tau, kappa, x), np.linalg.solve(A, x)) < 1e-12
    assert rel(orc.solve_seq2(scheme, nx, ny, ell, tau, kappa, x, transpose=True),
               np.linalg.solve(A.T, x)) < 1e-12
    for tr in (False, True):
        z, ratio = orc.pinv2_direct(scheme, nx, ny, ell, tau, kappa, x, transpose=tr)
        assert rel(z, np.linalg.solve(C.T if tr else C, x)) < 1e-11 and ratio < 1e-12
    u0, v0 = x[:nx * ny], x[nx * ny:2 * nx * ny]
    b = orc.build_rhs2(scheme, nx, ny, ell, tau, kappa, u0, v0 if scheme == BD2 else None)
    if scheme == HEAT:
        assert rel(b[0], M2 @ u0) < 1e-14 and np.all(b[1:] == 0)
    else:
        assert rel(b[0], (M2 + tau * tau * kappa * K2) @ (u0 + tau * v0)) < 1e-14
        assert rel(b[1], -M2 @ u0) < 1e-14 and np.all(b[2:] == 0)


def test_2d_heat_preconditioned_structure(orc):
    """A - C is the wrapped corner block (time row 0, column ell - 1), so C^{-1} A - I
    vanishes on every column but those of the last time level, where it equals
    C^{-1} applied to M2 placed in time row 0 (the negated wrapped block -M2)."""
    nx, ny, ell = 3, 2, 6
    tau = 1.0 / ell
    nn = nx * ny
    N = nn * ell
    I = np.eye(N)
    M2, _ = dense_MK2(nx, ny)
    D = np.column_stack([orc.pinv2_direct(HEAT, nx, ny, ell, tau, 1.0,
                                          orc.apply_A2(HEAT, nx, ny, ell, tau, 1.0, I[:, c]))[0].ravel()
                         for c in range(N)]) - I
    assert np.max(np.abs(D[:, :N - nn])) < 1e-13
    for c in range(nn):
        e = np.zeros((ell, nn))
        e[0] = M2[:, c]
        ref = orc.pinv2_direct(HEAT, nx, ny, ell, tau, 1.0, e)[0].ravel()
        assert rel(D[:, N - nn + c], ref) < 1e-12


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
@pytest.mark.parametrize("transpose", [False, True])
def test_2d_pinv_matches_eigendecomposition(orc, scheme, transpose):
    """The oracle's 2D C^{-1} (direct DFT in time, banded 2D solves) against the full
    eigen-decomposition of the block circulant (FFT in time, sine transforms along y
    and x, division by alpha_j mu_pq + beta_j kappa lambda_pq), every scheme."""
    nx, ny, ell = 6, 4, 7
    tau, kappa = 1.0 / ell, 0.7
    r = np.random.default_rng([70, scheme]).standard_normal((ell, nx * ny))
    z, _ = orc.pinv2_direct(scheme, nx, ny, ell, tau, kappa, r, transpose=transpose)
    ref = pins.pinv_spectral2(scheme, nx, ny, ell, tau, kappa, r, transpose)
    tol = max(1e-13, 8 * 2.0 ** -52 * pins.cond_C2(scheme, nx, ny, ell, tau, kappa))
    assert rel(z, ref) < tol


@pytest.mark.parametrize("scheme", [2, 3])
def test_2d_bd4_cd_rhs_by_sine_modes(orc, scheme):
    """BD4 (system C_BD4) and central differences (eq. CenDiffDisc) on the unit square:
    every block is a combination of M2 and K2, which act on the sine product s_q (x) s_p
    as mu_pq and lambda_pq mu_pq (lambda_pq = lambda^x_p + lambda^y_q).  Per mode, BD4 is
    the scalar recursion c_1 = c_0 + tau d_0, (1 + t) c_2 = 2 c_1 - c_0, (2 + t) c_k =
    5 c_{k-1} - 4 c_{k-2} + c_{k-3} (t = tau^2 kappa lambda_pq), and CD the ell x ell
    tridiagonal system c_{k-1} + (t - 2) c_k + c_{k+1} = 0 with c_0 moved to the right.
    The oracle's right-hand side solved by block substitution must give these modes."""
    nx, ny, ell, kappa = 7, 5, 9, 1.3
    tau = 1.0 / ell
    rng = np.random.default_rng(63)
    Sx = np.sin(np.pi * np.outer(np.arange(1, nx + 1), np.arange(1, nx + 1)) / (nx + 1))
    Sy = np.sin(np.pi * np.outer(np.arange(1, ny + 1), np.arange(1, ny + 1)) / (ny + 1))
    C0 = rng.standard_normal((ny, nx))
    D0 = rng.standard_normal((ny, nx))
    u0 = (Sy.T @ C0 @ Sx).ravel()
    v0 = (Sy.T @ D0 @ Sx).ravel() if scheme == 2 else None
    b = orc.build_rhs2(scheme, nx, ny, ell, tau, kappa, u0, v0)
    if scheme == 2:
        U = orc.solve_seq2(scheme, nx, ny, ell, tau, kappa, b)
    else:
        # CD couples u_{k+1} into row k, so no block substitution: solve with the
        # matrix that the oracle's matvec applies, column by column
        N = nx * ny * ell
        A = np.stack([orc.apply_A2(scheme, nx, ny, ell, tau, kappa, e).ravel()
                      for e in np.eye(N)], axis=1)
        U = np.linalg.solve(A, b.ravel()).reshape(ell, nx * ny)
    lam = pins.lam(ny, np.arange(1, ny + 1))[:, None] + pins.lam(nx, np.arange(1, nx + 1))[None, :]
    t = tau * tau * kappa * lam
    if scheme == 2:
        c = [C0, C0 + tau * D0]
        c.append((2 * c[1] - c[0]) / (1 + t))
        for k in range(3, ell + 1):
            c.append((5 * c[k - 1] - 4 * c[k - 2] + c[k - 3]) / (2 + t))
        modes = c[1:]
    else:
        modes = np.empty((ell, ny, nx))
        for q in range(ny):
            for p in range(nx):
                T = (np.diag(np.full(ell, t[q, p] - 2.0)) + np.eye(ell, k=1)
                     + np.eye(ell, k=-1))
                rhs = np.zeros(ell)
                rhs[0] = -C0[q, p]
                modes[:, q, p] = np.linalg.solve(T, rhs)
    for k in range(ell):
        assert rel(U[k], (Sy.T @ modes[k] @ Sx).ravel()) < 1e-11


def test_2d_rhs_rejections(orc):
    u0 = np.ones(12)
    with pytest.raises(RuntimeError):
        orc.build_rhs2(2, 4, 3, 2, 0.5, 1.0, u0)          # BD4 needs ell >= 3
    with pytest.raises(RuntimeError):
        orc.build_rhs2(1, 4, 3, 1, 0.5, 1.0, u0)          # BD2 needs ell >= 2
    with pytest.raises(RuntimeError):
        orc.build_rhs2(3, 4, 3, 4, 0.25, 1.0, u0, u0)     # CD takes no velocity
