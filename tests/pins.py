"""Independent mathematics used to pin the oracle (closed forms, quadrature,
dense Kronecker assembly).  Nothing here calls the oracle or the GPU library."""
import numpy as np
from scipy import integrate


def hat(i, n):
    """P1 hat function of interior node i (1-based) on the uniform mesh."""
    h = 1.0 / (n + 1)
    xi = i * h

    def phi(x):
        return max(0.0, 1.0 - abs(x - xi) / h)
    return phi, xi - h, xi + h


def quad_MK(n):
    """M_ij = int phi_i phi_j, K_ij = int phi_i' phi_j' by adaptive quadrature
    (element by element, so the kinks sit on interval ends)."""
    h = 1.0 / (n + 1)
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    for i in range(1, n + 1):
        for j in range(max(1, i - 1), min(n, i + 1) + 1):
            pi, a, b = hat(i, n)
            pj, _, _ = hat(j, n)
            lo = max(a, (j - 1) * h)
            hi = min(b, (j + 1) * h)
            if hi <= lo:
                continue
            nodes = np.arange(0, n + 2) * h
            pts = [p for p in nodes if lo < p < hi]
            edges = [lo] + pts + [hi]
            mv = 0.0
            kv = 0.0
            for e0, e1 in zip(edges[:-1], edges[1:]):
                mv += integrate.quad(lambda x: pi(x) * pj(x), e0, e1, epsabs=1e-15, epsrel=1e-13)[0]
                mid = 0.5 * (e0 + e1)
                di = (1.0 / h) * (1 if mid < i * h else -1)
                dj = (1.0 / h) * (1 if mid < j * h else -1)
                kv += di * dj * (e1 - e0)
            M[i - 1, j - 1] = mv
            K[i - 1, j - 1] = kv
    return M, K


def sine_vec(n, m):
    h = 1.0 / (n + 1)
    return np.sin(m * np.pi * h * np.arange(1, n + 1))


def mu(n, m):
    """Eigenvalue of M on sine mode m."""
    h = 1.0 / (n + 1)
    return (h / 3.0) * (2.0 + np.cos(m * np.pi * h))


def lam(n, m):
    """Generalised eigenvalue of (K, M) on sine mode m."""
    h = 1.0 / (n + 1)
    c = np.cos(m * np.pi * h)
    return 6.0 * (1.0 - c) / (h * h * (2.0 + c))


def sine_coeffs(u):
    """Coefficients c_m with u = sum_m c_m s_m (discrete sine transform, DST-I)."""
    n = u.size
    h = 1.0 / (n + 1)
    i = np.arange(1, n + 1)
    S = np.sin(np.pi * h * np.outer(np.arange(1, n + 1), i))
    return (2.0 / (n + 1)) * S @ u


def sine_synth(c):
    n = c.size
    h = 1.0 / (n + 1)
    i = np.arange(1, n + 1)
    S = np.sin(np.pi * h * np.outer(np.arange(1, n + 1), i))
    return S.T @ c


def heat_closed_form(u0, ell, tau, kappa):
    """u_k = sum_m c_m (1 + tau kappa lambda_m)^{-k} s_m, k = 1..ell."""
    n = u0.size
    c = sine_coeffs(u0)
    m = np.arange(1, n + 1)
    fac = 1.0 / (1.0 + tau * kappa * lam(n, m))
    U = np.empty((ell, n))
    ck = c.copy()
    for k in range(ell):
        ck = ck * fac
        U[k] = sine_synth(ck)
    return U


def bd2_closed_form(u0, v0, ell, tau, kappa):
    """Per sine mode the BD2 recursion (1 + tau^2 kappa lambda) c_k - 2 c_{k-1} + c_{k-2} = 0
    with c_0 = u_0 mode, c_1 = c_0 + tau d_0 has c_k = rho^k (c_0 cos k phi + B sin k phi),
    rho = (1 + tau^2 kappa lambda)^{-1/2}, phi = atan(tau sqrt(kappa lambda))."""
    n = u0.size
    c0 = sine_coeffs(u0)
    d0 = sine_coeffs(v0) if v0 is not None else np.zeros(n)
    m = np.arange(1, n + 1)
    lm = lam(n, m)
    rho = 1.0 / np.sqrt(1.0 + tau * tau * kappa * lm)
    phi = np.arctan(tau * np.sqrt(kappa * lm))
    c1 = c0 + tau * d0
    B = (c1 / rho - c0 * np.cos(phi)) / np.sin(phi)
    U = np.empty((ell, n))
    for k in range(1, ell + 1):
        ck = rho ** k * (c0 * np.cos(k * phi) + B * np.sin(k * phi))
        U[k - 1] = sine_synth(ck)
    return U


def bd4_mode_recursion(u0, v0, ell, tau, kappa):
    """Per sine mode (blocks act as mu, lambda mu on mode m) the BD4 system C_BD4 is the
    scalar recursion c_1 = c_0 + tau d_0 (start-up row), (1 + tau^2 kappa lambda) c_2 -
    2 c_1 + c_0 = 0 (BD2 row), (2 + tau^2 kappa lambda) c_k - 5 c_{k-1} + 4 c_{k-2} -
    c_{k-3} = 0 for k >= 3."""
    n = u0.size
    c0 = sine_coeffs(u0)
    d0 = sine_coeffs(v0) if v0 is not None else np.zeros(n)
    lm = lam(n, np.arange(1, n + 1))
    t2 = tau * tau * kappa * lm
    c = [c0, c0 + tau * d0]
    c.append((2 * c[1] - c[0]) / (1 + t2))
    for k in range(3, ell + 1):
        c.append((5 * c[k - 1] - 4 * c[k - 2] + c[k - 3]) / (2 + t2))
    return np.array([sine_synth(ck) for ck in c[1:ell + 1]])


def cd_mode_solve(u0, ell, tau, kappa):
    """Per sine mode the central-difference system C_CD is the ell x ell tridiagonal
    Toeplitz system c_{k-1} + (tau^2 kappa lambda - 2) c_k + c_{k+1} = 0, k = 1..ell,
    with c_0 the mode of u_0 moved to the right and no c_{ell+1} (the common factor mu
    cancels)."""
    n = u0.size
    c0 = sine_coeffs(u0)
    lm = lam(n, np.arange(1, n + 1))
    C = np.empty((ell, n))
    for m in range(n):
        T = (np.diag(np.full(ell, tau * tau * kappa * lm[m] - 2.0)) + np.eye(ell, k=1)
             + np.eye(ell, k=-1))
        rhs = np.zeros(ell)
        rhs[0] = -c0[m]
        C[:, m] = np.linalg.solve(T, rhs)
    return np.array([sine_synth(ck) for ck in C])


def kron_A(blocks, ell, circulant=False):
    """sum_m Shift^m (x) A_m with Shift the ell x ell down-shift (cyclic if circulant)."""
    n = blocks[0].shape[0]
    A = np.zeros((n * ell, n * ell))
    for m, B in enumerate(blocks):
        S = np.eye(ell, k=-m)
        if circulant and m > 0:
            S = S + np.eye(ell, k=ell - m)
        A += np.kron(S, B)
    return A


def alpha_beta(scheme, ell, tau, transpose=False):
    """Symbols alpha_j = sum_m a_m w^{jm}, beta_j = sum_m b_m w^{jm} of the circulant
    (blocks a_m M + b_m kappa K), w = exp(-+2 pi i / ell), in closed form."""
    j = np.arange(ell)
    w = np.exp((1j if transpose else -1j) * 2 * np.pi * j / ell)
    if scheme == 0:
        al, be = 1 - w, np.full(ell, tau)
    elif scheme == 1:
        al, be = (1 - w) ** 2, np.full(ell, tau * tau)
    elif scheme == 2:                       # BD4: 2 - 5 w + 4 w^2 - w^3 = (1 - w)^2 (2 - w)
        al, be = (1 - w) ** 2 * (2 - w), np.full(ell, tau * tau)
    else:                                   # CD: w^{-1} - 2 + w = -4 sin^2(pi j / ell)
        al, be = -4.0 * np.sin(np.pi * j / ell) ** 2 + 0j, np.full(ell, tau * tau)
    return al, be


def eig_C(scheme, n, ell, tau, kappa, transpose=False):
    """Eigenvalues of the block circulant on the (frequency j, sine mode m) basis:
    hatA_j = alpha_j M + beta_j kappa K acts on sine mode m as
    alpha_j mu_m + beta_j kappa lambda_m mu_m (M, K share the sine eigenvectors)."""
    h = 1.0 / (n + 1)
    m = np.arange(1, n + 1)
    c = np.cos(m * np.pi * h)
    mu_ = (h / 3.0) * (2.0 + c)
    lam_ = 6.0 * (1.0 - c) / (h * h * (2.0 + c))
    al, be = alpha_beta(scheme, ell, tau, transpose)
    return al[:, None] * mu_[None, :] + be[:, None] * kappa * (lam_ * mu_)[None, :]


def cond_C(scheme, n, ell, tau, kappa):
    e = np.abs(eig_C(scheme, n, ell, tau, kappa))
    return e.max() / e.min()


def pinv_spectral(scheme, n, ell, tau, kappa, r, transpose=False):
    """C^{-1} r through the full eigen-decomposition of the block circulant: FFT in
    time, DST-I in space, division by the eigenvalues, inverse transforms.  Its
    rounding error does not grow with cond(hatA_j) the way an elimination's does,
    so it is the accuracy reference for ill-conditioned symbols."""
    from scipy.fft import dst, idst
    X = np.fft.fft(np.asarray(r, dtype=np.float64).reshape(ell, n), axis=0)
    Xs = dst(X, type=1, axis=1)
    Ys = Xs / eig_C(scheme, n, ell, tau, kappa, transpose)
    Y = idst(Ys, type=1, axis=1)
    return np.fft.ifft(Y, axis=0).real


def eig_C2(scheme, nx, ny, ell, tau, kappa, transpose=False):
    """Eigenvalues of the 2D block circulant (Q1 blocks alpha_j M2 + beta_j kappa K2)
    on the (frequency j, sine mode q in y, sine mode p in x) basis, shape (ell, ny, nx):
    M2 and K2 = Ky (x) Mx + My (x) Kx share the sine-product eigenvectors, with the 1D
    eigenvalues mu (mass) and lambda mu (stiffness) along each axis."""
    def mk(n):
        h = 1.0 / (n + 1)
        c = np.cos(np.arange(1, n + 1) * np.pi * h)
        mu_ = (h / 3.0) * (2.0 + c)
        return mu_, 2.0 * (1.0 - c) / h
    mux, kx = mk(nx)
    muy, ky = mk(ny)
    m2 = muy[:, None] * mux[None, :]
    k2 = ky[:, None] * mux[None, :] + muy[:, None] * kx[None, :]
    al, be = alpha_beta(scheme, ell, tau, transpose)
    return al[:, None, None] * m2[None] + be[:, None, None] * kappa * k2[None]


def cond_C2(scheme, nx, ny, ell, tau, kappa):
    e = np.abs(eig_C2(scheme, nx, ny, ell, tau, kappa))
    return e.max() / e.min()


def pinv_spectral2(scheme, nx, ny, ell, tau, kappa, r, transpose=False):
    """2D C^{-1} r by the full eigen-decomposition: FFT in time, DST-I along y and x,
    division by the eigenvalues, inverse transforms."""
    from scipy.fft import dstn, idstn
    X = np.fft.fft(np.asarray(r, dtype=np.float64).reshape(ell, ny, nx), axis=0)
    Xs = dstn(X, type=1, axes=(1, 2))
    Y = idstn(Xs / eig_C2(scheme, nx, ny, ell, tau, kappa, transpose), type=1, axes=(1, 2))
    return np.fft.ifft(Y, axis=0).real
