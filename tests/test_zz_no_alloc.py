"""The allocation-free preconditioner apply (aao_apply_Pinv_noalloc) against the
context-based aao_apply_Pinv, both called through the C ABI: calls in a row on the
shared static scratch, each with a smaller input than the one before (and another
scheme, precision and orientation), each checked against the context path and
against the oracle; sizes beyond the static array are rejected before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HEAT, BD2 = 0, 1
FP64, MIXED, MIXED_IN = 0, 1, 3
UNSUPPORTED = -6


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_1810_00615_amd._lib import lib
    return lib()


def ctx_pinv(L, n, ell, tau, kappa, scheme, prec, r, transpose, stream):
    import torch
    ctx = ctypes.c_void_p()
    assert L.aao_create(n, ell, tau, scheme, ctypes.byref(ctx)) == 0
    try:
        assert L.aao_set_stream(ctx, ctypes.c_void_p(stream)) == 0
        assert L.aao_set_kappa(ctx, kappa) == 0
        assert L.aao_set_precision(ctx, prec) == 0
        z = torch.empty_like(r)
        assert L.aao_apply_Pinv(ctx, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                0, transpose) == 0
        torch.cuda.synchronize()
    finally:
        L.aao_destroy(ctx)
    return z


def noalloc_pinv(L, n, ell, tau, kappa, scheme, prec, r, transpose, stream):
    import torch
    z = torch.full_like(r, float("nan"))
    st = L.aao_apply_Pinv_noalloc(n, ell, tau, kappa, scheme, prec, ctypes.c_void_p(r.data_ptr()),
                                  ctypes.c_void_p(z.data_ptr()), transpose, ctypes.c_void_p(stream))
    assert st == 0, st
    torch.cuda.synchronize()
    return z


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_noalloc_matches_context_apply_twice(L, orc):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    cases = [  # (n, ell, kappa, scheme, precision, transpose, tolerance vs context, vs oracle)
        (1023, 1024, 1.3, HEAT, FP64, 0, 1e-14, 1e-10),
        (63, 64, 0.8, BD2, MIXED, 1, 1e-14, 2e-5),
        (31, 32, 1.1, HEAT, MIXED_IN, 0, 1e-14, 1e-5),
    ]
    for k, (n, ell, kappa, scheme, prec, tr, tol_ctx, tol_orc) in enumerate(cases):
        tau = 1.0 / ell
        print(f"case {k}: n={n} ell={ell} scheme={scheme} prec={prec} transpose={tr}", flush=True)
        rr = np.random.default_rng([31, k]).standard_normal((ell, n))
        r = torch.from_numpy(rr).cuda()
        z_na = noalloc_pinv(L, n, ell, tau, kappa, scheme, prec, r, tr, stream)
        z_cx = ctx_pinv(L, n, ell, tau, kappa, scheme, prec, r, tr, stream)
        assert bool(torch.isfinite(z_na).all())
        e_ctx = rel(z_na.cpu().numpy(), z_cx.cpu().numpy())
        e_orc = rel(z_na.cpu().numpy(), orc.pinv(scheme, n, ell, tau, kappa, rr, transpose=bool(tr)))
        print(f"  vs context {e_ctx:.2e}, vs oracle {e_orc:.2e}")
        assert e_ctx <= tol_ctx
        assert e_orc <= tol_orc


def test_noalloc_rejects_oversize(L):
    import torch
    r = torch.zeros(16, dtype=torch.float64, device="cuda")
    z = torch.zeros(16, dtype=torch.float64, device="cuda")
    # n = 8191, ell = 8192 in FP64 needs about 538 MB of scratch: rejected on the host
    st = L.aao_apply_Pinv_noalloc(8191, 8192, 1.0 / 8192, 1.0, HEAT, FP64,
                                  ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()), 0,
                                  None)
    assert st == UNSUPPORTED
    # a length that is not a power of two
    st = L.aao_apply_Pinv_noalloc(3, 5, 0.2, 1.0, HEAT, FP64, ctypes.c_void_p(r.data_ptr()),
                                  ctypes.c_void_p(z.data_ptr()), 0, None)
    assert st == UNSUPPORTED
