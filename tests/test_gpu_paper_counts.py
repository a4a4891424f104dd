"""The paper-table regression suite on the GPU path: every printed GMRES iteration
count of Tables 1, 3(a), 4 and 5 (tolerance 1e-5; fixture tests/golden/
paper_iteration_counts.txt) is reproduced by the library's right-preconditioned
FGMRES from x0 = 0, and by the library's operators in the paper's left-preconditioned
form.

The paper uses left preconditioning and does not state its norm or counting
convention, so each count is compared within the slack of the oracle's own
left-preconditioned pin (one iteration; two for the one printed outlier), and the
GPU count is compared with the oracle's right-preconditioned FGMRES on the same
input within one iteration (its stopping test is also the estimate, confirmed by
the true residual; rounding can move a count that sits at the tolerance by one)."""
import numpy as np
import pytest

from test_oracle_paper_tables import SLACK, rows

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("row", rows(), ids=lambda r: f"{r[0]}-{r[1]}-{r[2]}x{r[3]}")
def test_gpu_iteration_counts(orc, row):
    import torch
    from paper_1810_00615_amd import Problem
    from paper_1810_00615_amd.inputs import paper_initial_data
    scheme_name, data, n, ell, printed = row
    scheme = 0 if scheme_name == "heat" else 1
    tau = 1.0 / ell
    u0 = paper_initial_data(data, n)
    P = Problem(n, ell, scheme="heat" if scheme == 0 else "bd2", kappa=1.0)
    b = P.rhs(torch.as_tensor(u0, dtype=torch.float64, device="cuda"))
    x, info = P.solve(b, restart=30, tol=1e-5, maxit=300)
    torch.cuda.synchronize()
    br = orc.build_rhs(scheme, n, ell, tau, 1.0, u0)
    xo, io = orc.fgmres(lambda v: orc.apply_A(scheme, n, ell, tau, 1.0, v.reshape(ell, n)).ravel(),
                        lambda v: orc.pinv(scheme, n, ell, tau, 1.0, v.reshape(ell, n)).ravel(),
                        br, 30, 1e-5, 300)
    X = x.cpu().numpy()
    res = np.linalg.norm(br - orc.apply_A(scheme, n, ell, tau, 1.0, X)) / np.linalg.norm(br)
    print(f"{scheme_name} {data} n={n} ell={ell}: printed {printed}, GPU {info['iters']}, "
          f"oracle (right) {io['iters']}, true residual {res:.1e}")
    assert info["status"] == 0 and res <= 1e-5
    assert abs(info["iters"] - io["iters"]) <= 1
    assert abs(info["iters"] - printed) <= SLACK.get((scheme_name, data, n, ell), 1)
    P.close()


@pytest.mark.parametrize("row", rows(), ids=lambda r: f"{r[0]}-{r[1]}-{r[2]}x{r[3]}")
def test_gpu_operators_left_counts(orc, row):
    """The paper's own form on the GPU operators: the library's matvec and C^{-1} inside
    left-preconditioned GMRES (C^{-1} A U = C^{-1} b from 0, relative 1e-5, counted in
    preconditioner applies after the initial one) give the oracle's left-preconditioned
    count (within one: rounding can move a count whose last residual sits at the
    tolerance) and stay within the printed count's slack."""
    import torch
    from test_oracle_paper_tables import initial
    from paper_1810_00615_amd import Problem
    scheme_name, data, n, ell, printed = row
    scheme = 0 if scheme_name == "heat" else 1
    tau = 1.0 / ell
    P = Problem(n, ell, scheme="heat" if scheme == 0 else "bd2", kappa=1.0)
    to = lambda v: torch.as_tensor(np.ascontiguousarray(v).reshape(ell, n), device="cuda")
    op = lambda v: P.Pinv(P.A(to(v))).cpu().numpy().ravel()
    b = orc.build_rhs(scheme, n, ell, tau, 1.0, initial(data, n)).ravel()
    bp = P.Pinv(to(b)).cpu().numpy().ravel()
    x, info = orc.fgmres(op, lambda v: v, bp, restart=100, tol=1e-5, maxit=100)
    opo = lambda v: orc.pinv(scheme, n, ell, tau, 1.0, orc.apply_A(scheme, n, ell, tau, 1.0, v)).ravel()
    bpo = orc.pinv(scheme, n, ell, tau, 1.0, b).ravel()
    xo, io = orc.fgmres(opo, lambda v: v, bpo, restart=100, tol=1e-5, maxit=100)
    print(f"{scheme_name} {data} n={n} ell={ell}: printed {printed}, GPU operators (left) "
          f"{info['iters']}, oracle (left) {io['iters']}")
    # a count whose last residual sits at the tolerance can move by one with rounding
    assert info["converged"] and abs(info["iters"] - io["iters"]) <= 1
    assert abs(info["iters"] - printed) <= SLACK.get((scheme_name, data, n, ell), 1)
    P.close()


@pytest.mark.parametrize("delta", [0.1, 0.9])
def test_gpu_table2_neumann_counts(orc, delta):
    """Table 2 on the GPU path (sub-table (a): n = 320, ell = 768): the library's
    variable-step matvec and Neumann preconditioner (orders 0..2) inside the
    left-preconditioned GMRES of the reading of Table 2 reproduce every printed count
    within one iteration; the library's own right-preconditioned FGMRES on the same grid
    converges to 1e-5 in the oracle's right-preconditioned count (within one)."""
    import torch
    from test_oracle_paper_tables import table2_count, table2_rows
    from paper_1810_00615_amd import Problem
    from paper_1810_00615_amd.inputs import paper_initial_data, perturbed_steps
    row = [r for r in table2_rows() if r[0] == "a" and r[3] == delta][0]
    _, n, ell, _, printed = row
    tau = 1.0 / ell
    for q in range(3):
        tk = perturbed_steps(ell, delta, [7, q])
        P = Problem(n, ell, tau, "heat", steps=tk, neumann_order=q)
        to = lambda v: torch.as_tensor(np.ascontiguousarray(v).reshape(ell, n), device="cuda")
        A = lambda v: P.A(to(v)).cpu().numpy().ravel()
        Pi = lambda v: P.Pinv(to(v), order=q).cpu().numpy().ravel()
        c, _ = table2_count(orc, n, ell, delta, q, [7, q], apply_op=A, apply_prec=Pi)
        b = P.rhs(torch.as_tensor(paper_initial_data("bump", n), device="cuda"))
        x, info = P.solve(b, restart=30, tol=1e-5, maxit=100)
        br = b.cpu().numpy().ravel()
        xo, io = orc.fgmres(lambda v: orc.apply_A(0, n, ell, tau, 1.0, v, tau_k=tk).ravel(),
                            lambda v: orc.neumann(0, n, ell, tau, 1.0, tk, v, q).ravel(),
                            br, 30, 1e-5, 100)
        print(f"table 2 (a) delta={delta} i={q + 1}: printed {printed[q]}, GPU operators "
              f"(left) {c}, GPU FGMRES (right) {info['iters']}, oracle (right) {io['iters']}")
        assert abs(c - printed[q]) <= 1
        assert info["converged"] and abs(info["iters"] - io["iters"]) <= 1
        P.close()
