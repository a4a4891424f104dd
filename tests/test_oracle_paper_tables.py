"""Loose pins against the iteration counts the paper prints (Tables 1, 4, 5).

The paper states the tolerance (1e-5) and left preconditioning but not the norm,
initial guess or how iterations are counted, so each count is matched within one
iteration.  Counting one iteration per preconditioner apply from x0 = 0, the
heat count comes out one lower than printed and the wave counts match."""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_iteration_counts.txt")


def rows():
    out = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        out.append((f[0], f[1], int(f[2]), int(f[3]), int(f[4])))
    return out


def initial(name, n):
    x = np.arange(1, n + 1) / (n + 1)
    if name == "x(1-x)":
        return x * (1 - x)
    if name == "sin2pix":
        return np.sin(2 * np.pi * x)
    return np.where((x > 3 / 8) & (x < 5 / 8), np.cos(4 * np.pi * (x - 0.5)) ** 2, 0.0)


@pytest.mark.parametrize("row", rows(), ids=lambda r: f"{r[0]}-{r[1]}-{r[2]}x{r[3]}")
def test_left_preconditioned_iteration_counts(orc, row):
    scheme_name, data, n, ell, printed = row
    scheme = 0 if scheme_name == "heat" else 1
    tau = 1.0 / ell
    b = orc.build_rhs(scheme, n, ell, tau, 1.0, initial(data, n)).ravel()
    op = lambda v: orc.pinv(scheme, n, ell, tau, 1.0, orc.apply_A(scheme, n, ell, tau, 1.0, v)).ravel()
    bp = orc.pinv(scheme, n, ell, tau, 1.0, b).ravel()
    x, info = orc.fgmres(op, lambda v: v, bp, restart=100, tol=1e-5, maxit=100)
    assert info["converged"]
    assert abs(info["iters"] - printed) <= 1
    U = orc.solve_seq(scheme, n, ell, tau, 1.0, b)
    assert np.linalg.norm(x - U.ravel()) / np.linalg.norm(U) < 1e-4
