"""The paper-table regression suite on the GPU path: every printed GMRES iteration
count of Tables 1, 3(a), 4 and 5 (tolerance 1e-5; fixture tests/golden/
paper_iteration_counts.txt) is reproduced by the library's right-preconditioned
FGMRES from x0 = 0.

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
