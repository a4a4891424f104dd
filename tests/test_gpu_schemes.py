"""The four-step backward-difference (BD4) and central-difference (CD) wave schemes
on the GPU against the oracle: right-hand sides, the matvec with its start-up rows
(BD4) or its block above the diagonal (CD) in both orientations, the circulant
preconditioner apply (power-of-two and Bluestein lengths, both orientations, against
the oracle and the eigen-decomposition reference), GMRES to the exact solution,
and the adjoint gradients.

Tolerances: right-hand side and matvec 1e-14 relative to the largest entry; C^{-1}
max(1e-10, 4 eps kappa_2(C)) (both schemes have nearly singular frequency blocks:
BD4 at j = 0, CD wherever 4 sin^2(pi j / ell) approaches tau^2 lambda_m); solutions
within max(1e-10, 4 kappa_2(A) tol) of the exact sequential solution."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BD4, CD = 2, 3
NAME = {BD4: "bd4", CD: "cd"}
EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def maxrel(a, b):
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


def normrel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def td(dev, x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(dev)


@pytest.mark.parametrize("scheme", [BD4, CD])
@pytest.mark.parametrize("n,ell", [(1, 3), (7, 5), (63, 64), (257, 100)])
def test_rhs(dev, orc, scheme, n, ell):
    from paper_1810_00615_amd import Problem
    tau, kappa = 1.0 / ell, 1.3
    rng = np.random.default_rng([n, ell, scheme])
    u0, v0 = rng.standard_normal(n), rng.standard_normal(n)
    P = Problem(n, ell, tau, NAME[scheme], kappa=kappa, device=dev)
    vv = v0 if scheme == BD4 else None
    b = P.rhs(td(dev, u0), None if vv is None else td(dev, vv)).cpu().numpy()
    ref = orc.build_rhs(scheme, n, ell, tau, kappa, u0, vv)
    assert maxrel(b, ref) < 1e-14
    if scheme == CD:
        from paper_1810_00615_amd import AAOError
        with pytest.raises(AAOError):
            P.rhs(td(dev, u0), td(dev, v0))


@pytest.mark.parametrize("scheme", [BD4, CD])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("n,ell", [(1, 1), (1, 4), (5, 3), (64, 17), (65, 9), (130, 33),
                                   (257, 100), (320, 9), (513, 24), (4097, 5)])
def test_apply_A(dev, orc, scheme, transpose, n, ell):
    from paper_1810_00615_amd import Problem
    tau, kappa = 1.0 / ell, 0.9
    x = np.random.default_rng([n, ell, 2]).standard_normal((ell, n))
    P = Problem(n, ell, tau, NAME[scheme], kappa=kappa, device=dev)
    y = P.A(td(dev, x), transpose=transpose).cpu().numpy()
    assert maxrel(y, orc.apply_A(scheme, n, ell, tau, kappa, x, transpose=transpose)) < 1e-14


@pytest.mark.parametrize("scheme", [BD4, CD])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("n,ell", [(1, 2), (5, 3), (63, 64), (127, 96), (255, 256), (4095, 16),
                                   (33, 1531)])
def test_pinv(dev, orc, scheme, transpose, n, ell):
    import pins
    from paper_1810_00615_amd import Problem
    tau, kappa = 1.0 / ell, 1.0
    r = np.random.default_rng([n, ell, 3]).standard_normal((ell, n))
    P = Problem(n, ell, tau, NAME[scheme], kappa=kappa, device=dev)
    z = P.Pinv(td(dev, r), transpose=transpose).cpu().numpy()
    tol = max(1e-10, 4 * EPS * pins.cond_C(scheme, n, ell, tau, kappa))
    e_orc = normrel(z, orc.pinv(scheme, n, ell, tau, kappa, r, transpose=transpose))
    e_spec = normrel(z, pins.pinv_spectral(scheme, n, ell, tau, kappa, r, transpose))
    print(f"{NAME[scheme]} pinv n={n} ell={ell} tr={transpose}: vs oracle {e_orc:.2e}, "
          f"vs spectral {e_spec:.2e}, tol {tol:.2e}")
    assert e_orc < tol and e_spec < tol


def test_bd4_gmres_bump_to_exact(dev, orc):
    """BD4 with the paper's non-smooth initial data u_0^{ns} (n = 64, ell = 96): FGMRES
    to 1e-10 reaches the exact sequential BD4 solution (the per-mode BD4 recursion pins
    that solution in the CPU tests)."""
    from paper_1810_00615_amd import Problem
    from paper_1810_00615_amd.inputs import paper_initial_data
    n, ell = 64, 96
    tau = 1.0 / ell
    u0 = paper_initial_data("bump", n)
    P = Problem(n, ell, tau, "bd4", device=dev)
    b = P.rhs(td(dev, u0))
    U, info = P.solve(b, restart=60, tol=1e-10, maxit=600)
    print(f"bd4 bump n={n} ell={ell}: iterations {info['iters']}, true {info['rel_resid_true']:.2e}")
    assert info["converged"]
    Ur = orc.solve_seq(BD4, n, ell, tau, 1.0, orc.build_rhs(BD4, n, ell, tau, 1.0, u0))
    # kappa_2(A) = 1.66e4 here (per-mode singular values of the BD4 recursion)
    assert normrel(U.cpu().numpy(), Ur) < 4 * 1.66e4 * 1e-10


def test_cd_gmres_smooth_two_iterations(dev, orc):
    """Central differences with the smooth u_0^{s2} = sin(2 pi x): the preconditioned
    system converges in two iterations (the count the paper reports for this data) and
    the solution is the exact block-tridiagonal one."""
    from paper_1810_00615_amd import Problem
    from paper_1810_00615_amd.inputs import paper_initial_data
    n, ell = 63, 64
    tau = 1.0 / ell
    u0 = paper_initial_data("sin2pix", n)
    P = Problem(n, ell, tau, "cd", device=dev)
    b = P.rhs(td(dev, u0))
    U, info = P.solve(b, restart=30, tol=1e-5, maxit=100)
    assert info["converged"] and info["iters"] <= 2
    U2, info2 = P.solve(b, restart=30, tol=1e-11, maxit=100)
    assert info2["converged"]
    Ur = orc.solve_seq(CD, n, ell, tau, 1.0, orc.build_rhs(CD, n, ell, tau, 1.0, u0))
    # kappa_2(A) = 5.4e4 here (per-mode eigenvalues mu (tau^2 lambda - 2 + 2 cos(pi k/(ell+1))))
    assert normrel(U2.cpu().numpy(), Ur) < 4 * 5.4e4 * 1e-11


@pytest.mark.parametrize("scheme", [BD4, CD])
def test_adjoint_gradients(dev, orc, scheme):
    """Gradients through autograd (transposed solve with C^{-T}, then the reductions)
    against the oracle's exact adjoint gradient."""
    import torch
    from paper_1810_00615_amd import Problem, all_at_once_solve
    n, ell, kappa = 31, 48, 1.2
    tau = 1.0 / ell
    rng = np.random.default_rng(50 + scheme)
    u0r = rng.standard_normal(n) * 0.1
    v0r = rng.standard_normal(n) * 0.1 if scheme == BD4 else None
    Ut = rng.standard_normal((ell, n)) * 0.01
    P = Problem(n, ell, tau, NAME[scheme], kappa=kappa, device=dev)
    u0 = td(dev, u0r).requires_grad_(True)
    v0 = td(dev, v0r).requires_grad_(True) if v0r is not None else None
    k = torch.tensor(kappa, dtype=torch.float64, device=dev, requires_grad=True)
    U = all_at_once_solve(u0, k, P, restart=60, tol=1e-13, maxit=1200, v0=v0)
    (0.5 * ((U - td(dev, Ut)) ** 2).sum()).backward()
    Ur = orc.solve_seq(scheme, n, ell, tau, kappa, orc.build_rhs(scheme, n, ell, tau, kappa, u0r, v0r))
    lr = orc.adjoint_seq(scheme, n, ell, tau, kappa, Ur - Ut)
    gur, gvr, gkr = orc.grad(scheme, n, ell, tau, kappa, u0r, Ur, lr, v0=v0r)
    e_u = normrel(u0.grad.cpu().numpy(), gur)
    e_k = abs(float(k.grad) - gkr) / abs(gkr)
    print(f"{NAME[scheme]} gradients: g_u0 {e_u:.2e}, g_kappa {e_k:.2e}")
    assert e_u < 1e-7 and e_k < 1e-7
    if v0 is not None:
        assert normrel(v0.grad.cpu().numpy(), gvr) < 1e-7
