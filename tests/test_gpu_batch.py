"""Batched form on the GPU: problems of uneven n and ell (including lengths with
large prime factors, ell = 2 and 3, n = 1) in one launch per phase, against the
oracle problem by problem; hipGraph replay against eager launches; the 64-problem
batch workload to 1e-8."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HEAT = 0
SMALL = [(63, 100), (255, 256), (17, 97), (400, 513), (31, 1000), (5, 2), (1, 3), (130, 1021)]


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    return torch.device("cuda:0")


def normrel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def make(dev, prec, sizes=SMALL, kap_seed=0):
    from paper_1810_00615_amd import Batch
    rng = np.random.default_rng(kap_seed)
    ns = [s[0] for s in sizes]
    ells = [s[1] for s in sizes]
    kappas = rng.uniform(0.5, 2.0, len(sizes))
    return Batch(ns, ells, kappas, precision=prec, device=dev), ns, ells, kappas


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 2e-6), ("fp32", 1e-3),
                                      ("mixed_in", 2e-6)])
def test_batch_pinv(dev, orc, prec, tol):
    import torch
    B, ns, ells, kappas = make(dev, prec)
    rs = [np.random.default_rng([i, 1]).standard_normal((l, n)) for i, (n, l) in enumerate(zip(ns, ells))]
    z = B.Pinv(B.pack(rs))
    for i, (zv, r) in enumerate(zip(B.views(z), rs)):
        ref = orc.pinv(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i], r)
        e = normrel(zv.cpu().numpy(), ref)
        print(f"batch pinv {prec} n={ns[i]} ell={ells[i]}: {e:.2e}")
        assert e < tol


LARGE = [(4095, 2048), (33, 1025), (700, 1531), (1, 1100)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 2e-6)])
def test_batch_pinv_long(dev, orc, prec, tol):
    """Bluestein lengths M = 4096 (ell 1025..2048): one column pair per workgroup,
    ragged last tiles (odd n, n = 1), the largest n."""
    B, ns, ells, kappas = make(dev, prec, sizes=LARGE, kap_seed=4)
    rs = [np.random.default_rng([i, 9]).standard_normal((l, n)) for i, (n, l) in enumerate(zip(ns, ells))]
    z = B.Pinv(B.pack(rs))
    for i, (zv, r) in enumerate(zip(B.views(z), rs)):
        ref = orc.pinv(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i], r)
        e = normrel(zv.cpu().numpy(), ref)
        print(f"batch pinv {prec} n={ns[i]} ell={ells[i]}: {e:.2e}")
        assert e < tol


def test_batch_matvec(dev, orc):
    B, ns, ells, kappas = make(dev, "mixed")
    xs = [np.random.default_rng([i, 2]).standard_normal((l, n)) for i, (n, l) in enumerate(zip(ns, ells))]
    y = B.A(B.pack(xs))
    for i, (yv, x) in enumerate(zip(B.views(y), xs)):
        ref = orc.apply_A(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i], x)
        assert float(np.max(np.abs(yv.cpu().numpy() - ref)) / np.max(np.abs(ref))) < 1e-14


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
def test_batch_gmres_small(dev, orc, prec):
    """Every member reaches the 1e-8 true residual (oracle FP64 matvec) and the exact
    sequential solution; graph replay gives bitwise the same result as eager launches."""
    B, ns, ells, kappas = make(dev, prec)
    J = 20
    modes = np.arange(1, J + 1)
    amps = np.random.default_rng(3).normal(0, 0.1, (len(ns), J))
    u0 = B.project_sine(modes, amps)
    b = B.rhs(u0)
    B.set_graph(True)
    x_g, infos, st = B.solve(b, restart=30, tol=1e-8, maxit=300)
    B.set_graph(False)
    x_e, infos_e, st_e = B.solve(b, restart=30, tol=1e-8, maxit=300)
    assert st == 0 and st_e == 0
    # (x0 = 0 by the zero-guess entry: the alignment padding between members is
    # never written, so compare the members' views)
    for vg, ve in zip(B.views(x_g), B.views(x_e)):
        assert bool((vg == ve).all())
    bcpu = [v.cpu().numpy() for v in B.views(b)]
    for i, (xv, bv) in enumerate(zip(B.views(x_g), bcpu)):
        n, ell, kap = ns[i], ells[i], kappas[i]
        u0r = orc.project_sine(n, modes.astype(np.int32), amps[i])
        br = orc.build_rhs(HEAT, n, ell, 1.0 / ell, kap, u0r)
        assert float(np.max(np.abs(bv - br)) / np.max(np.abs(br))) < 1e-12
        X = xv.cpu().numpy()
        res = np.linalg.norm(br - orc.apply_A(HEAT, n, ell, 1.0 / ell, kap, X)) / np.linalg.norm(br)
        U = orc.solve_seq(HEAT, n, ell, 1.0 / ell, kap, br)
        print(f"batch gmres {prec} n={n} ell={ell}: iters {infos[i]['iters']} res {res:.2e} "
              f"err {normrel(X, U):.2e}")
        assert infos[i]["converged"] and res <= 1e-8
        assert normrel(X, U) < 1e-6


@pytest.mark.parametrize("restart", [30, 2])
def test_batch_zero_guess(dev, orc, restart):
    """The zero-guess entry (first cycle starts from b itself, x only written: the
    output buffer starts as NaN) matches an explicit zero initial guess, also when
    the problems restart, and every member meets the 1e-8 true residual (oracle FP64
    matvec); an all-zero right-hand side returns x = 0.  (The two entries sum |b|^2
    in different orders, so they agree to rounding, not bitwise.)"""
    import torch
    B, ns, ells, kappas = make(dev, "fp64")
    J = 20
    modes = np.arange(1, J + 1)
    amps = np.random.default_rng(5).normal(0, 0.1, (len(ns), J))
    b = B.rhs(B.project_sine(modes, amps))
    out = torch.full((B.total,), float("nan"), dtype=torch.float64, device=dev)
    x_z, inf_z, st_z = B.solve(b, restart=restart, tol=1e-8, maxit=300, out=out)
    x_e, inf_e, st_e = B.solve(b, restart=restart, tol=1e-8, maxit=300, x0=B.zeros())
    torch.cuda.synchronize()
    print(f"zero guess restart {restart}: iterations {[i['iters'] for i in inf_z]} "
          f"(explicit {[i['iters'] for i in inf_e]}) status {st_z}")
    assert st_z == 0 and st_e == 0
    bcpu = [v.cpu().numpy() for v in B.views(b)]
    # (the alignment padding between members belongs to no problem: compare the views)
    for i, (vz, ve, bv) in enumerate(zip(B.views(x_z), B.views(x_e), bcpu)):
        X = vz.cpu().numpy()
        res = np.linalg.norm(bv - orc.apply_A(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i], X)) \
            / np.linalg.norm(bv)
        assert res <= 1e-8, (i, res)
        if inf_z[i]["iters"] == inf_e[i]["iters"]:
            assert normrel(X, ve.cpu().numpy()) < 1e-12
        else:
            assert abs(inf_z[i]["iters"] - inf_e[i]["iters"]) <= 1
            assert normrel(X, ve.cpu().numpy()) < 1e-6
    out.fill_(float("nan"))
    x0, inf0, st0 = B.solve(B.zeros(), restart=restart, tol=1e-8, maxit=300, out=out)
    assert st0 == 0 and all(bool((v == 0).all()) for v in B.views(x0))


@pytest.mark.parametrize("restart", [30, 2, 1])
def test_batch_delayed_matches_classic(dev, orc, restart):
    """CGS2 with the re-orthogonalisation deferred by one step (two passes per step)
    against the three-pass form (AAO_GMRES_CGS2_CLASSIC): the same iteration counts and the
    same solutions to rounding, with and without restarts; both meet the 1e-8 true
    residual (oracle FP64 matvec)."""
    import torch
    J = 20
    modes = np.arange(1, J + 1)
    amps = np.random.default_rng(6).normal(0, 0.1, (len(SMALL), J))
    out = {}
    for name in ("delayed", "classic"):
        B, ns, ells, kappas = make(dev, "fp64")
        b = B.rhs(B.project_sine(modes, amps))
        x, infos, st = B.solve(b, restart=restart, tol=1e-8, maxit=300, cgs2=name)
        torch.cuda.synchronize()
        assert st == 0
        out[name] = ([v.cpu().numpy() for v in B.views(x)], [i["iters"] for i in infos],
                     [v.cpu().numpy() for v in B.views(b)])
        B.close()
    xd, itd, bd = out["delayed"]
    xc, itc, _ = out["classic"]
    print(f"restart {restart}: iterations delayed {itd} classic {itc}")
    for i, (a, c, bv) in enumerate(zip(xd, xc, bd)):
        res = np.linalg.norm(bv - orc.apply_A(HEAT, SMALL[i][0], SMALL[i][1], 1.0 / SMALL[i][1],
                                              make_kappas()[i], a)) / np.linalg.norm(bv)
        assert res <= 1e-8, (i, res)
        assert abs(itd[i] - itc[i]) <= 1
        if itd[i] == itc[i]:
            assert normrel(a, c) < 1e-10


@pytest.mark.parametrize("restart", [8, 30])
def test_batch_delayed_bd2_long(dev, orc, restart):
    """Many Arnoldi steps and restarts (wave BD2, 20-mode data): the deferred and the
    three-pass CGS2 both reach the 1e-8 true residual (oracle FP64 BD2 matvec) with
    iteration counts within two of each other."""
    import torch
    from paper_1810_00615_amd import Batch
    sizes = [(63, 64), (127, 256), (31, 100)]
    ns = [a for a, _ in sizes]
    ells = [c for _, c in sizes]
    modes = np.arange(1, 21)
    amps = np.random.default_rng(8).normal(0, 0.1, (len(sizes), 20))
    its = {}
    for name in ("delayed", "classic"):
        B = Batch(ns, ells, [1.0] * len(sizes), scheme="bd2", precision="fp64", device=dev)
        b = B.rhs(B.project_sine(modes, amps))
        x, infos, st = B.solve(b, restart=restart, tol=1e-8, maxit=400, cgs2=name)
        torch.cuda.synchronize()
        assert st == 0
        for i, (xv, bv) in enumerate(zip(B.views(x), B.views(b))):
            X, bb = xv.cpu().numpy(), bv.cpu().numpy()
            res = np.linalg.norm(bb - orc.apply_A(1, ns[i], ells[i], 1.0 / ells[i], 1.0, X)) \
                / np.linalg.norm(bb)
            assert res <= 1e-8, (name, i, res)
        its[name] = [i["iters"] for i in infos]
        B.close()
    print(f"BD2 restart {restart}: iterations delayed {its['delayed']} classic {its['classic']}")
    for a, c in zip(its["delayed"], its["classic"]):
        assert abs(a - c) <= 2


def make_kappas(kap_seed=0):
    return np.random.default_rng(kap_seed).uniform(0.5, 2.0, len(SMALL))


def test_batch_rejects_overlap(dev):
    """b and x sharing memory is an argument error (x is written while b is read)."""
    from paper_1810_00615_amd._lib import AAOError
    B, ns, ells, kappas = make(dev, "fp64")
    b = B.rhs(B.project_sine(np.arange(1, 4), np.ones((len(ns), 3))))
    with pytest.raises(AAOError):
        B.solve(b, out=b)
    with pytest.raises(AAOError):
        B.solve(b, x0=b, out=b)


def test_batch_transpose_solve(dev, orc):
    """transpose=True solves A_p^T x_p = b_p to the 1e-8 true residual (oracle FP64
    transposed matvec) for every member."""
    B, ns, ells, kappas = make(dev, "fp64")
    gs = [np.random.default_rng([i, 7]).standard_normal((l, n)) for i, (n, l) in enumerate(zip(ns, ells))]
    x, infos, st = B.solve(B.pack(gs), restart=30, tol=1e-8, maxit=300, transpose=True)
    assert st == 0
    for i, (xv, g) in enumerate(zip(B.views(x), gs)):
        X = xv.cpu().numpy()
        res = np.linalg.norm(g - orc.apply_A(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i], X,
                                             transpose=True)) / np.linalg.norm(g)
        print(f"batch transpose n={ns[i]} ell={ells[i]}: iters {infos[i]['iters']} res {res:.2e}")
        assert infos[i]["converged"] and res <= 1e-8


def test_batch_mixed_in_solve(dev, orc):
    """Input-side single precision in the batch: every member meets the 1e-8 true residual
    (oracle FP64 matvec) in at most one iteration more than the FP64 batch (the
    single-precision rounding of the input side leaves a relative residual of a few
    units of 1e-8 after the first iteration, so members that FP64 finishes in one
    iteration take two)."""
    J = 20
    modes = np.arange(1, J + 1)
    amps = np.random.default_rng(16).normal(0, 0.1, (len(SMALL), J))
    its = {}
    for prec in ("fp64", "mixed_in"):
        B, ns, ells, kappas = make(dev, prec)
        b = B.rhs(B.project_sine(modes, amps))
        x, infos, st = B.solve(b, restart=30, tol=1e-8, maxit=300)
        assert st == 0, prec
        for i, (xv, bv) in enumerate(zip(B.views(x), B.views(b))):
            bb = bv.cpu().numpy()
            res = np.linalg.norm(bb - orc.apply_A(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i],
                                                  xv.cpu().numpy())) / np.linalg.norm(bb)
            assert infos[i]["converged"] and res <= 1e-8, (prec, i, res)
        its[prec] = [i["iters"] for i in infos]
        B.close()
    print("batch iterations:", its)
    for a, b64 in zip(its["mixed_in"], its["fp64"]):
        assert a <= max(b64, 2)


def test_batch_forward_then_transpose_same_batch(dev, orc):
    """A forward solve and then a transposed solve on the same Batch with graph replay
    on (the captured steps depend on the orientation and must be recaptured), then a
    forward solve again: each meets the 1e-8 true residual of its own operator."""
    B, ns, ells, kappas = make(dev, "fp64")
    B.set_graph(True)
    gs = [np.random.default_rng([i, 8]).standard_normal((l, n)) for i, (n, l) in enumerate(zip(ns, ells))]
    g = B.pack(gs)
    for tr in (False, True, False):
        x, infos, st = B.solve(g, restart=30, tol=1e-8, maxit=300, transpose=tr)
        assert st == 0, tr
        for i, (xv, gv) in enumerate(zip(B.views(x), gs)):
            res = np.linalg.norm(gv - orc.apply_A(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i],
                                                  xv.cpu().numpy(), transpose=tr)) / np.linalg.norm(gv)
            assert infos[i]["converged"] and res <= 1e-8, (tr, i, res)


def test_batch_workload_64(dev, orc):
    """The 64-problem batch (n in U{255..4095}, ell in U{256..2048}, kappa in U[0.5, 2],
    20-mode u0): single-precision transforms, FP64 outer FGMRES(30) to 1e-8, every member
    checked by the oracle's FP64 matvec and exact time stepping."""
    from paper_1810_00615_amd import Batch
    from paper_1810_00615_amd.inputs import heat_batch
    ws = heat_batch()
    B = Batch([w.n for w in ws], [w.ell for w in ws], [w.kappa for w in ws], precision="mixed",
              device=dev)
    modes = ws[0].modes
    amps = np.stack([w.amps for w in ws])
    u0 = B.project_sine(modes, amps)
    b = B.rhs(u0)
    x, infos, st = B.solve(b, restart=30, tol=1e-8, maxit=300)
    assert st == 0
    worst = 0.0
    for i, (xv, w) in enumerate(zip(B.views(x), ws)):
        u0r = orc.project_sine(w.n, w.modes, w.amps)
        br = orc.build_rhs(HEAT, w.n, w.ell, w.tau, w.kappa, u0r)
        X = xv.cpu().numpy()
        res = np.linalg.norm(br - orc.apply_A(HEAT, w.n, w.ell, w.tau, w.kappa, X)) / np.linalg.norm(br)
        worst = max(worst, res)
        assert infos[i]["converged"] and res <= 1e-8, (i, w.n, w.ell, res)
    print(f"batch 64: max true residual {worst:.2e}, iterations "
          f"{sorted(set(i['iters'] for i in infos))}")


def test_batch_graph_spans_match_eager(dev, orc):
    """Arnoldi steps captured per step, per three steps and per whole restart cycle (one
    graph launch per cycle), and launched eagerly: bitwise the same solutions and the
    same iteration counts (steps after convergence run fully masked), with restarts."""
    J = 20
    modes = np.arange(1, J + 1)
    amps = np.random.default_rng(17).normal(0, 0.1, (len(SMALL), J))
    res = {}
    B, ns, ells, kappas = make(dev, "fp64")
    b = B.rhs(B.project_sine(modes, amps))
    for name, graph, span in (("eager", False, 1), ("span1", True, 1), ("span3", True, 3),
                              ("cycle", True, 0)):
        B.set_graph(graph)
        B.set_config("graph_span", span)
        x, infos, st = B.solve(b, restart=5, tol=1e-9, maxit=300)
        assert st == 0, name
        # members only: with the zero guess the alignment padding is never written
        res[name] = ([v.cpu().numpy() for v in B.views(x)], [i["iters"] for i in infos])
    print("iterations:", res["eager"][1])
    for name in ("span1", "span3", "cycle"):
        assert res[name][1] == res["eager"][1], name
        for a, e in zip(res[name][0], res["eager"][0]):
            assert np.array_equal(a, e), name


@pytest.mark.parametrize("slab,rows", [(1024, 2), (16384, 8), (256, 4)])
def test_batch_shapes_parity(dev, orc, slab, rows):
    """Other slab sizes and matvec tile heights: the matvec (both orientations) against the
    oracle and a solve to the 1e-8 true residual."""
    B, ns, ells, kappas = make(dev, "fp64")
    B.set_config("slab", slab)
    B.set_config("matvec_rows", rows)
    assert B.configs()["slab"] == slab and B.configs()["matvec_rows"] == rows
    xs = [np.random.default_rng([i, 5]).standard_normal((l, n)) for i, (n, l) in enumerate(zip(ns, ells))]
    for tr in (False, True):
        y = B.A(B.pack(xs), transpose=tr)
        for i, (yv, xv) in enumerate(zip(B.views(y), xs)):
            ref = orc.apply_A(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i], xv, transpose=tr)
            assert np.max(np.abs(yv.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
    b = B.pack(xs)
    x, infos, st = B.solve(b, restart=30, tol=1e-8, maxit=300)
    assert st == 0
    for i, (xv, bv) in enumerate(zip(B.views(x), xs)):
        r = bv - orc.apply_A(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i], xv.cpu().numpy())
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(bv)


def test_batch_tune_picks_admissible_shapes(dev, orc, tmp_path):
    """The batch tuner times the slab sizes, matvec tile heights and (given a right-hand
    side) graph spans on the batch's own sizes, keeps admissible ones, writes them to the
    tuning file, and a second batch of the same sizes takes them from the cache."""
    from paper_1810_00615_amd.api import set_tune_cache
    cache = tmp_path / "btune.txt"
    set_tune_cache(str(cache))
    try:
        J = 20
        modes = np.arange(1, J + 1)
        amps = np.random.default_rng(18).normal(0, 0.1, (len(SMALL), J))
        B, ns, ells, kappas = make(dev, "mixed_in")
        b = B.rhs(B.project_sine(modes, amps))
        cfg = B.tune(b, restart=30, tol=1e-8, maxit=300, reps=2)
        print("tuned batch shapes:", cfg)
        assert cfg["slab"] in (1024, 2048, 4096, 8192, 16384)
        assert cfg["matvec_rows"] in (2, 4, 8)
        assert cfg["graph_span"] in (1, 2, 4, 0)
        assert len(cache.read_text().splitlines()) == 3
        B2, *_ = make(dev, "mixed_in")
        assert B2.tune(b, reps=2) == cfg
        assert len(cache.read_text().splitlines()) == 3
        x, infos, st = B2.solve(b, restart=30, tol=1e-8, maxit=300)
        assert st == 0
        for i, (xv, bv) in enumerate(zip(B2.views(x), B2.views(b))):
            bb = bv.cpu().numpy()
            r = bb - orc.apply_A(HEAT, ns[i], ells[i], 1.0 / ells[i], kappas[i], xv.cpu().numpy())
            assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(bb)
    finally:
        set_tune_cache(None)
