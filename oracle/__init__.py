"""CPU FP64 oracle for the all-at-once circulant-preconditioned GMRES path.

TEST INFRASTRUCTURE.  Only the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1810_00615_amd``) and never imports it.

What the oracle computes, and the passage of Goddard & Wathen (arXiv
1810.00615) each function follows:

* ``apply_A`` / ``solve_seq`` / ``adjoint_seq`` -- the monolithic systems of
  Sec. 2: eq. monolithicheat for heat, the systems C_BD2 and C_BD4 (two start-up
  rows) and the two-sided central-difference system C_CD for the wave equation,
  eq. nonuniformmonolithicheat with variable steps.  ``solve_seq`` is forward block
  substitution, i.e. the sequential time stepping the monolithic system packages
  (for C_CD, Gaussian elimination with partial pivoting on its band): the exact
  solution U.
* ``apply_C`` -- the block circulant preconditioner (eq. standardheatprecon,
  eq. wavepreconditioner, R_BD4, R_CD).
* ``dft`` -- the direct O(ell^2) transform along time (the (U (x) I_n) factor of
  eq. precon2para in the per-column form of eq. alternativecal).
* ``pinv_direct`` / ``pinv`` -- C^{-1} r by the Fourier diagonalisation of
  eq. precon2para: transform, one complex tridiagonal (Thomas) solve per
  frequency (Sec. 3), inverse transform.  ``pinv`` uses numpy's FFT as the
  transform step (a library primitive) and is pinned to ``pinv_direct``.
* ``neumann`` -- the truncated Neumann series of eq. preconapprox1 for the
  variable-step preconditioner Q = P + sigma (x) K.
* ``fgmres`` -- textbook restarted right-preconditioned (flexible) GMRES with
  modified Gram-Schmidt and Givens rotations (Saad & Schultz, cited in Sec. 1).
* ``grad`` -- adjoint-gradient reductions for d/du_0 and d/dkappa.

Readings of the paper (M + tau K for the printed K + tau M, n = interior nodes,
L2 projection of the initial data, ...) are the ones listed in the design notes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HEAT = 0
BD2 = 1
BD4 = 2
CD = 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aao_oracle.c")
_SRC2 = os.path.join(_HERE, "aao_oracle2d.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (plain -O2, OpenMP for the
    loops over independent columns / frequencies)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
             _SRC, _SRC2, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                   os.path.getmtime(_SRC2)):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        for name in ("or_scheme_coeffs", "or_toeplitz", "or_block", "or_load_sine",
                     "or_project_sine", "or_build_rhs",
                     "or_solve_seq", "or_adjoint_seq", "or_apply_A", "or_apply_C", "or_apply_E",
                     "or_shifted_solve_all", "or_pinv_direct", "or_grad", "or_mk_solve",
                     "or2_mk_solve", "or2_apply_A", "or2_apply_C", "or2_solve_seq",
                     "or2_build_rhs", "or2_pinv_direct"):
            getattr(lib, name).restype = ctypes.c_int
        for name in ("or_dft", "or_mass_apply", "or_stiff_apply", "or_symbol", "or2_mk_apply"):
            getattr(lib, name).restype = None
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _chk(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


# ------------------------------------------------------------------ space

def mass(n, x):
    x = _c(x)
    y = np.empty(n)
    _load().or_mass_apply(n, _p(x), _p(y))
    return y


def stiff(n, x):
    x = _c(x)
    y = np.empty(n)
    _load().or_stiff_apply(n, _p(x), _p(y))
    return y


def mk_solve(n, cm, ck, r):
    """Solve (cm M + ck K) x = r by the Thomas algorithm."""
    r = _c(r)
    x = np.empty(n)
    _chk(_load().or_mk_solve(n, ctypes.c_double(cm), ctypes.c_double(ck), _p(r), _p(x)),
         "mk_solve")
    return x


def toeplitz(scheme, tau):
    """(mlo, a, b): the Toeplitz blocks a_m M + b_m kappa K of the scheme for offsets
    m = mlo .. mlo + len(a) - 1 (block (k, k - m) of the monolithic matrix)."""
    a = np.zeros(4)
    b = np.zeros(4)
    mlo = ctypes.c_int(0)
    mhi = ctypes.c_int(0)
    if _load().or_toeplitz(scheme, ctypes.c_double(tau), ctypes.byref(mlo), ctypes.byref(mhi),
                           _p(a), _p(b)) != 0:
        raise ValueError("unknown scheme")
    k = mhi.value - mlo.value + 1
    return mlo.value, a[:k].copy(), b[:k].copy()


def block(scheme, ell, tau, kappa, k, m, tau_k=None):
    """(cm, ck) of the block in row k, column k - m (cm M + ck K), or None."""
    cm = ctypes.c_double(0.0)
    ck = ctypes.c_double(0.0)
    tk = None if tau_k is None else _c(tau_k)
    ok = _load().or_block(scheme, ctypes.c_double(tau), ctypes.c_double(kappa),
                          _p(tk) if tk is not None else None, ell, k, m, ctypes.byref(cm),
                          ctypes.byref(ck))
    return (cm.value, ck.value) if ok else None


def load_sine(n, modes, amps):
    modes = np.ascontiguousarray(modes, dtype=np.int32)
    amps = _c(amps)
    f = np.empty(n)
    _load().or_load_sine(n, len(modes), modes.ctypes.data_as(_ip), _p(amps), _p(f))
    return f


def project_sine(n, modes, amps):
    """u_0 = M^{-1} f, the L2 projection of sum_m amps[m] sin(modes[m] pi x)."""
    modes = np.ascontiguousarray(modes, dtype=np.int32)
    amps = _c(amps)
    u0 = np.empty(n)
    _chk(_load().or_project_sine(n, len(modes), modes.ctypes.data_as(_ip), _p(amps), _p(u0)),
         "project_sine")
    return u0


# -------------------------------------------------------------- monolithic

def build_rhs(scheme, n, ell, tau, kappa, u0, v0=None):
    u0 = _c(u0)
    v0p = _p(_c(v0)) if v0 is not None else None
    b = np.empty((ell, n))
    _chk(_load().or_build_rhs(scheme, n, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                              _p(u0), v0p, _p(b)), "build_rhs")
    return b


def _tk(tau_k):
    return None if tau_k is None else _p(_c(tau_k))


def apply_A(scheme, n, ell, tau, kappa, x, transpose=False, tau_k=None):
    x = _c(x).reshape(ell, n)
    tk = None if tau_k is None else _c(tau_k)
    y = np.empty((ell, n))
    _chk(_load().or_apply_A(scheme, n, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                            _p(tk) if tk is not None else None, _p(x), _p(y), int(transpose)),
         "apply_A")
    return y


def apply_C(scheme, n, ell, tau, kappa, x, transpose=False):
    x = _c(x).reshape(ell, n)
    y = np.empty((ell, n))
    _chk(_load().or_apply_C(scheme, n, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                            _p(x), _p(y), int(transpose)), "apply_C")
    return y


def apply_E(n, ell, tau, kappa, tau_k, x):
    x = _c(x).reshape(ell, n)
    tk = _c(tau_k)
    y = np.empty((ell, n))
    _chk(_load().or_apply_E(n, ell, ctypes.c_double(tau), ctypes.c_double(kappa), _p(tk),
                            _p(x), _p(y)), "apply_E")
    return y


def _cd_banded(n, ell, tau, kappa):
    """The central-difference matrix C_CD (eq. CenDiffDisc: M u_{k-1} + (tau^2 kappa K
    - 2M) u_k + M u_{k+1}, no u_{ell+1}) in LAPACK band storage, l = u = n + 1:
    ab[u + r - c, c] = A[r, c] with r = k n + i, c = k' n + j."""
    h = 1.0 / (n + 1)
    N = n * ell
    w = n + 1
    ab = np.zeros((2 * w + 1, N))

    def put(r, c, v):
        ab[w + r - c, c] += v
    t2 = tau * tau * kappa
    for k in range(ell):
        for dk, (cm, ck) in ((-1, (1.0, 0.0)), (0, (-2.0, t2)), (1, (1.0, 0.0))):
            kk = k + dk
            if not 0 <= kk < ell:
                continue
            for i in range(n):
                r = k * n + i
                put(r, kk * n + i, cm * 4.0 * h / 6.0 + ck * 2.0 / h)
                if i > 0:
                    put(r, kk * n + i - 1, cm * h / 6.0 - ck / h)
                if i < n - 1:
                    put(r, kk * n + i + 1, cm * h / 6.0 - ck / h)
    return ab, w


def _cd_solve(n, ell, tau, kappa, rhs):
    """Exact solution of the symmetric system C_CD X = rhs: Gaussian elimination with
    partial pivoting on its band (LAPACK gbsv through scipy, a library solve)."""
    from scipy.linalg import solve_banded
    ab, w = _cd_banded(n, ell, tau, kappa)
    return solve_banded((w, w), ab, _c(rhs).ravel()).reshape(ell, n)


def solve_seq(scheme, n, ell, tau, kappa, b, tau_k=None):
    """Exact U with A U = b by forward block substitution (time stepping); for the
    two-sided central-difference system a banded solve with partial pivoting."""
    if scheme == CD:
        if tau_k is not None:
            raise ValueError("variable steps are defined for the heat scheme only")
        return _cd_solve(n, ell, tau, kappa, b)
    b = _c(b).reshape(ell, n)
    tk = None if tau_k is None else _c(tau_k)
    U = np.empty((ell, n))
    _chk(_load().or_solve_seq(scheme, n, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                              _p(tk) if tk is not None else None, _p(b), _p(U)), "solve_seq")
    return U


def adjoint_seq(scheme, n, ell, tau, kappa, g, tau_k=None):
    """Exact L with A^T L = g by backward block substitution (central differences:
    C_CD is symmetric, so the banded solve of solve_seq)."""
    if scheme == CD:
        return solve_seq(scheme, n, ell, tau, kappa, g, tau_k)
    g = _c(g).reshape(ell, n)
    tk = None if tau_k is None else _c(tau_k)
    L = np.empty((ell, n))
    _chk(_load().or_adjoint_seq(scheme, n, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                                _p(tk) if tk is not None else None, _p(g), _p(L)),
         "adjoint_seq")
    return L


# ----------------------------------------------------------------- Fourier

def dft(x, inverse=False):
    """Direct DFT along axis 0 of an ell x n (complex) array."""
    x = np.asarray(x)
    ell, n = x.shape
    xr = _c(x.real)
    xi = _c(x.imag) if np.iscomplexobj(x) else None
    Xr = np.empty((ell, n))
    Xi = np.empty((ell, n))
    _load().or_dft(ell, n, _p(xr), _p(xi) if xi is not None else None, _p(Xr), _p(Xi),
                   int(inverse))
    return Xr + 1j * Xi


def symbol(scheme, ell, tau, j, transpose=False):
    """(alpha_j, beta_j) with hatA_j = alpha_j M + beta_j kappa K."""
    out = np.empty(4)
    _load().or_symbol(scheme, ell, ctypes.c_double(tau), j, int(transpose), _p(out))
    return complex(out[0], out[1]), complex(out[2], out[3])


def shifted_solve_all(scheme, n, ell, tau, kappa, X, transpose=False):
    """Y_j = hatA_j^{-1} X_j for every row j of an ell x n complex array."""
    Xr = _c(np.real(X))
    Xi = _c(np.imag(X))
    _chk(_load().or_shifted_solve_all(scheme, n, ell, ctypes.c_double(tau),
                                      ctypes.c_double(kappa), int(transpose), _p(Xr), _p(Xi)),
         "shifted_solve_all")
    return Xr + 1j * Xi


def pinv_direct(scheme, n, ell, tau, kappa, r, transpose=False):
    """C^{-1} r with the direct DFT (O(n ell^2)); returns (z, max|Im|/max|Re|)."""
    r = _c(r).reshape(ell, n)
    z = np.empty((ell, n))
    ratio = ctypes.c_double(0.0)
    _chk(_load().or_pinv_direct(scheme, n, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                                int(transpose), _p(r), _p(z), ctypes.byref(ratio)),
         "pinv_direct")
    return z, ratio.value


def pinv(scheme, n, ell, tau, kappa, r, transpose=False):
    """C^{-1} r with numpy's FFT as the transform step (same definition as
    ``pinv_direct``; numpy.fft.fft uses the kernel exp(-2 pi i jk/ell))."""
    r = _c(r).reshape(ell, n)
    X = np.fft.fft(r, axis=0)
    Y = shifted_solve_all(scheme, n, ell, tau, kappa, X, transpose)
    return np.ascontiguousarray(np.fft.ifft(Y, axis=0).real)


def neumann(scheme, n, ell, tau, kappa, tau_k, r, order, transpose=False, direct=False):
    """Truncated Neumann series of eq. preconapprox1,
    sum_{m=0}^{order} (-C^{-1} E)^m C^{-1} r, E = blockdiag((tau_k - tau) kappa K),
    evaluated by the recurrence z_0 = C^{-1} r, z_m = C^{-1}(r - E z_{m-1}).
    (E is block diagonal and symmetric, so the transposed series uses C^{-T}.)"""
    P = (lambda v: pinv_direct(scheme, n, ell, tau, kappa, v, transpose)[0]) if direct else \
        (lambda v: pinv(scheme, n, ell, tau, kappa, v, transpose))
    r = _c(r).reshape(ell, n)
    z = P(r)
    for _ in range(order):
        z = P(r - apply_E(n, ell, tau, kappa, tau_k, z))
    return z


# ------------------------------------------------------------------ GMRES

def fgmres(apply_op, apply_prec, b, restart, tol, maxit, x0=None):
    """Restarted right-preconditioned flexible GMRES (modified Gram-Schmidt,
    Givens rotations), stopping when the least-squares residual estimate
    |g_{j+1}| / ||b|| <= tol and confirming with the true residual
    ||b - A x|| / ||b|| before returning.  Counts preconditioner applies.

    Returns (x, info) with info = dict(iters, restarts, converged, est, true, hist)."""
    b = _c(b).ravel()
    N = b.size
    x = np.zeros(N) if x0 is None else _c(x0).ravel().copy()
    bnorm = np.linalg.norm(b)
    info = dict(iters=0, restarts=0, converged=False, est=np.nan, true=np.nan, hist=[])
    if bnorm == 0.0:
        x[:] = 0.0
        info.update(converged=True, est=0.0, true=0.0)
        return x, info
    r = b - apply_op(x)
    beta = np.linalg.norm(r)
    info["true"] = beta / bnorm
    if beta / bnorm <= tol:
        info.update(converged=True, est=beta / bnorm)
        return x, info
    while info["iters"] < maxit:
        m = restart
        V = np.zeros((m + 1, N))
        Z = np.zeros((m, N))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            Z[j] = apply_prec(V[j])
            w = apply_op(Z[j])
            info["iters"] += 1
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            est = abs(g[j + 1]) / bnorm
            info["hist"].append(est)
            info["est"] = est
            if est <= tol or info["iters"] >= maxit:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + Z[:k].T @ y
        r = b - apply_op(x)
        beta = np.linalg.norm(r)
        info["true"] = beta / bnorm
        if beta / bnorm <= tol:
            info["converged"] = True
            break
        info["restarts"] += 1
    return x, info


# --------------------------------------------------------------- gradient

def grad(scheme, n, ell, tau, kappa, u0, U, L, v0=None, tau_k=None):
    """(g_u0, g_v0, g_kappa) of L(U) given the adjoint solution L (A^T L = dL/dU)."""
    u0 = _c(u0)
    U = _c(U).reshape(ell, n)
    L = _c(L).reshape(ell, n)
    v0c = _c(v0) if v0 is not None else None
    tk = None if tau_k is None else _c(tau_k)
    gu = np.empty(n)
    gv = np.empty(n)
    gk = ctypes.c_double(0.0)
    _chk(_load().or_grad(scheme, n, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                         _p(tk) if tk is not None else None, _p(u0),
                         _p(v0c) if v0c is not None else None, _p(U), _p(L), _p(gu), _p(gv),
                         ctypes.byref(gk)), "grad")
    return gu, gv, gk.value


# ------------------------------------------------------- two space dimensions
# Q1 elements on the uniform nx x ny interior grid of the unit square: M2 = My (x) Mx,
# K2 = Ky (x) Mx + My (x) Kx; a time level is an (ny, nx) array, x fastest
# (aao_oracle2d.c).

def mk2(nx, ny, cm, ck, x):
    """(cm M2 + ck K2) x for one time level."""
    x = _c(x).reshape(ny, nx)
    y = np.empty((ny, nx))
    _load().or2_mk_apply(nx, ny, ctypes.c_double(cm), ctypes.c_double(ck), _p(x), _p(y))
    return y


def mk2_solve(nx, ny, cm, ck, r):
    r = _c(r).reshape(ny, nx)
    u = np.empty((ny, nx))
    _chk(_load().or2_mk_solve(nx, ny, ctypes.c_double(cm), ctypes.c_double(ck), _p(r), _p(u)),
         "mk2_solve")
    return u


def apply_A2(scheme, nx, ny, ell, tau, kappa, x, transpose=False):
    x = _c(x).reshape(ell, ny * nx)
    y = np.empty((ell, ny * nx))
    _chk(_load().or2_apply_A(scheme, nx, ny, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                             _p(x), _p(y), int(transpose)), "apply_A2")
    return y


def apply_C2(scheme, nx, ny, ell, tau, kappa, x, transpose=False):
    x = _c(x).reshape(ell, ny * nx)
    y = np.empty((ell, ny * nx))
    _chk(_load().or2_apply_C(scheme, nx, ny, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                             _p(x), _p(y), int(transpose)), "apply_C2")
    return y


def solve_seq2(scheme, nx, ny, ell, tau, kappa, b, transpose=False):
    """Exact U of the 2D monolithic system (A^T U = b with transpose) by block
    substitution in time."""
    b = _c(b).reshape(ell, ny * nx)
    U = np.empty((ell, ny * nx))
    _chk(_load().or2_solve_seq(scheme, nx, ny, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                               _p(b), _p(U), int(transpose)), "solve_seq2")
    return U


def build_rhs2(scheme, nx, ny, ell, tau, kappa, u0, v0=None):
    u0 = _c(u0).ravel()
    v0p = _p(_c(v0).ravel()) if v0 is not None else None
    b = np.empty((ell, ny * nx))
    _chk(_load().or2_build_rhs(scheme, nx, ny, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                               _p(u0), v0p, _p(b)), "build_rhs2")
    return b


def pinv2_direct(scheme, nx, ny, ell, tau, kappa, r, transpose=False):
    """C^{-1} r in 2D with the direct DFT and banded 2D solves; (z, max|Im|/max|Re|)."""
    r = _c(r).reshape(ell, ny * nx)
    z = np.empty((ell, ny * nx))
    ratio = ctypes.c_double(0.0)
    _chk(_load().or2_pinv_direct(scheme, nx, ny, ell, ctypes.c_double(tau), ctypes.c_double(kappa),
                                 int(transpose), _p(r), _p(z), ctypes.byref(ratio)), "pinv2_direct")
    return z, ratio.value
