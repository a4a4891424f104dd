"""Launch shapes and the autotuner on the GPU: every admissible shape of the forward
transform, the shifted solves and the inverse transform gives the oracle's C^{-1} r
(Sec. 3, eq. precon2para) to the same tolerance as the default shapes, and every
matvec shape the oracle's block-Toeplitz product (Sec. 2); aao_tune picks admissible
shapes, caches them per process and in the aao_set_tune_cache file, and the tuned apply still
matches the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HEAT, BD2 = 0, 1
EPS = 2.0 ** -52
FFT_CODES = list(range(0, 7)) + list(range(16, 23))


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def normrel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def admissible(P, kernel, codes):
    from paper_1810_00615_amd import AAOError
    out = []
    for c in codes:
        try:
            P.set_config(kernel, c)
        except AAOError:
            continue
        out.append(c)
    P.set_config(kernel, -1)
    return out


# (n, ell): several chunks and a ragged last chunk; ell from 64 to 2048, one size
# with n past 4096 (only wide chunks / many threads cover it)
SHAPES = [(1000, 256), (63, 64), (2047, 1024), (4500, 128), (130, 2048)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,ell", SHAPES)
def test_every_shape_matches_oracle(dev, orc, n, ell, prec):
    """FP64: 1e-10 relative up to n = 4096; beyond, the forward-error bound
    4 eps kappa_2(C) of an elimination without pivoting (the zero-frequency block is
    kappa tau K, whose condition number grows like n^2: about 8e6 at n = 4500)."""
    import torch
    import pins
    from paper_1810_00615_amd import Problem
    tau, kappa = 1.0 / ell, 1.1
    r = np.random.default_rng([n, ell, 11]).standard_normal((ell, n))
    ref = orc.pinv(HEAT, n, ell, tau, kappa, r)
    P = Problem(n, ell, tau, "heat", kappa=kappa, precision=prec, device=dev)
    rd = torch.from_numpy(r).to(dev)
    if prec == "fp64":
        tol = 1e-10 if n <= 4096 else max(1e-10, 4 * EPS * pins.cond_C(HEAT, n, ell, tau, kappa))
    else:
        tol = 2e-6
    solve_codes = admissible(P, "shifted_solve", range(64))
    assert solve_codes, "no solve shape admitted"
    fft_codes = admissible(P, "fft_fwd", FFT_CODES)
    assert fft_codes == admissible(P, "fft_inv", FFT_CODES)
    worst = {}
    for kernel, codes in (("shifted_solve", solve_codes), ("fft_fwd", fft_codes),
                          ("fft_inv", fft_codes)):
        for c in codes:
            P.set_config(kernel, c)
            e = normrel(P.Pinv(rd).cpu().numpy(), ref)
            worst[(kernel, c)] = e
            assert e < tol, (kernel, c, P.configs(), e)
        P.set_config(kernel, -1)
    print(f"n={n} ell={ell} {prec}: {len(solve_codes)} solve / {len(fft_codes)} fft shapes, "
          f"worst {max(worst.values()):.2e}")


def test_solve_shapes_bd2_transpose(dev, orc):
    """Indefinite BD2 symbols and the transposed (conjugated) symbol through every
    solve shape."""
    import torch
    import pins
    from paper_1810_00615_amd import Problem
    n, ell = 700, 512
    tau, kappa = 1.0 / ell, 1.0
    r = np.random.default_rng(12).standard_normal((ell, n))
    ref = orc.pinv(BD2, n, ell, tau, kappa, r, transpose=True)
    tol = max(1e-10, 4 * EPS * pins.cond_C(BD2, n, ell, tau, kappa))
    P = Problem(n, ell, tau, "bd2", kappa=kappa, device=dev)
    rd = torch.from_numpy(r).to(dev)
    for c in admissible(P, "shifted_solve", range(64)):
        P.set_config("shifted_solve", c)
        e = normrel(P.Pinv(rd, transpose=True).cpu().numpy(), ref)
        assert e < tol, (c, e, tol)


def test_tune_picks_admissible_shapes(dev, orc, tmp_path):
    import torch
    from paper_1810_00615_amd import Problem
    from paper_1810_00615_amd.api import set_tune_cache
    cache = tmp_path / "tune.txt"
    set_tune_cache(str(cache))
    n, ell = 1023, 512
    tau, kappa = 1.0 / ell, 0.9
    P = Problem(n, ell, tau, "heat", kappa=kappa, device=dev)
    cfg = P.tune(reps=3)
    print("tuned:", cfg)
    assert all(v is not None for v in cfg.values())
    code, (cw, nt, staged) = cfg["shifted_solve"]
    assert n <= cw * nt and staged in (0, 1)
    assert cfg["fft_fwd"][1][1] in (1, 2, 4, 8, 16, 32, 64)
    lines = cache.read_text().split()
    assert len(lines) == 4 * 6
    # a second context of the same size takes the cached shapes without timing
    Q = Problem(n, ell, tau, "heat", kappa=kappa, device=dev)
    assert Q.tune(reps=3) == cfg
    assert len(cache.read_text().split()) == 4 * 6
    r = np.random.default_rng(5).standard_normal((ell, n))
    z = Q.Pinv(torch.from_numpy(r).to(dev)).cpu().numpy()
    assert normrel(z, orc.pinv(HEAT, n, ell, tau, kappa, r)) < 1e-10
    # the tuned solve converges like the default one
    b = Q.rhs(Q.project_sine(np.arange(1, 6, dtype=np.int32), np.ones(5)))
    U, info = Q.solve(b, restart=30, tol=1e-10, maxit=100)
    assert info["converged"]
    ref = orc.solve_seq(HEAT, n, ell, tau, kappa, b.cpu().numpy())
    assert normrel(U.cpu().numpy(), ref) < 1e-8
    set_tune_cache(None)


MV_SHAPES = [(1, 1), (2, 3), (63, 5), (64, 17), (65, 16), (130, 33), (257, 100), (4095, 9)]


@pytest.mark.parametrize("scheme", [HEAT, BD2])
@pytest.mark.parametrize("n,ell", MV_SHAPES)
def test_matvec_every_shape(dev, orc, scheme, n, ell):
    """Every matvec launch shape (rows per thread 4/8/16, DPP or ds_bpermute lane
    moves), forward and transposed, against the oracle's block-Toeplitz product;
    widths around the 64-lane wave edges and time lengths around the row tiles."""
    import torch
    from paper_1810_00615_amd import Problem
    tau, kappa = 1.0 / ell, 0.8
    x = np.random.default_rng([n, ell, 13]).standard_normal((ell, n))
    P = Problem(n, ell, tau, "heat" if scheme == HEAT else "bd2", kappa=kappa, device=dev)
    xd = torch.from_numpy(x).to(dev)
    for tr in (False, True):
        ref = orc.apply_A(scheme, n, ell, tau, kappa, x, transpose=tr)
        for code in range(6):
            P.set_config("matvec", code)
            y = P.A(xd, transpose=tr).cpu().numpy()
            err = float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))
            assert err < 1e-14, (code, tr, err)


def test_matvec_shapes_variable_steps(dev, orc):
    import torch
    from paper_1810_00615_amd import Problem
    from paper_1810_00615_amd.inputs import perturbed_steps
    n, ell = 200, 37
    tk = perturbed_steps(ell, 0.7, [9, 1])
    x = np.random.default_rng(14).standard_normal((ell, n))
    P = Problem(n, ell, 1.0 / ell, "heat", kappa=1.3, steps=tk, device=dev)
    xd = torch.from_numpy(x).to(dev)
    for tr in (False, True):
        ref = orc.apply_A(HEAT, n, ell, 1.0 / ell, 1.3, x, transpose=tr, tau_k=tk)
        for code in range(6):
            P.set_config("matvec", code)
            y = P.A(xd, transpose=tr).cpu().numpy()
            assert float(np.max(np.abs(y - ref)) / np.max(np.abs(ref))) < 1e-14, (code, tr)


@pytest.mark.parametrize("code", [1, 4])
@pytest.mark.parametrize("scheme,restart", [(HEAT, 3), (BD2, 8)])
def test_solution_update_paths(dev, orc, code, scheme, restart):
    """The solution update and residual check in one launch (DPP launch shapes, at
    most four directions, zero initial guess) and as a separate update plus check
    (other shapes, more directions, restart cycles): both reach the requested true
    residual, and the reported residual is the oracle's."""
    import torch
    from paper_1810_00615_amd import Problem
    n, ell = 255, 128
    tau, kappa = 1.0 / ell, 1.0
    P = Problem(n, ell, tau, "heat" if scheme == HEAT else "bd2", kappa=kappa, device=dev)
    P.set_config("matvec", code)
    rng = np.random.default_rng([code, restart])
    br = np.zeros((ell, n))
    br[:2] = rng.standard_normal((2, n))
    b = torch.from_numpy(br).to(dev)
    U, info = P.solve(b, restart=restart, tol=1e-10, maxit=600)
    assert info["converged"], info
    Un = U.cpu().numpy()
    rel = np.linalg.norm(br - orc.apply_A(scheme, n, ell, tau, kappa, Un)) / np.linalg.norm(br)
    assert rel <= 1.0001e-10
    assert abs(info["rel_resid_true"] - rel) < 1e-12
