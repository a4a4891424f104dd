"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/aao.h declares, and rejects bad arguments before it
touches the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aao.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(aao_[A-Za-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_1810_00615_amd._lib import lib
    return lib()


def test_header_declares_the_boundary():
    names = declared()
    for required in ("aao_create", "aao_apply_A", "aao_apply_Pinv", "aao_gmres",
                     "aao_adjoint_solve", "aao_destroy", "aao_grad"):
        assert required in names


def test_every_declared_symbol_is_exported(L):
    for name in declared():
        assert hasattr(L, name), name


def test_binding_covers_every_symbol():
    from paper_1810_00615_amd._lib import SIGNATURES
    assert set(declared()) <= set(SIGNATURES), set(declared()) - set(SIGNATURES)


@pytest.mark.parametrize("args", [(0, 4, 0.1, 0), (4, 0, 0.1, 0), (4, 4, 0.0, 0),
                                  (4, 4, -1.0, 0), (4, 4, float("nan"), 0), (4, 4, 0.1, 7)])
def test_create_rejects_bad_arguments(L, args):
    c = ctypes.c_void_p()
    assert L.aao_create(*args, ctypes.byref(c)) == -1
    assert not c.value


@pytest.mark.parametrize("args,code", [((0, 3, 4, 0.1, 0), -1), ((4, 0, 4, 0.1, 0), -1),
                                       ((4, 3, 0, 0.1, 0), -1), ((4, 3, 4, 0.0, 0), -1),
                                       ((4, 3, 4, 0.1, 7), -1), ((4, 4, 4, 0.1, 0), -6),
                                       ((4, 6, 4, 0.1, 0), -6), ((4, 4095, 4, 0.1, 0), -6),
                                       ((20000, 3, 4, 0.1, 0), -6)])
def test_create_2d_rejects_bad_arguments(L, args, code):
    """Argument errors, and grids whose y size is not one below a power of two (the sine
    transform's requirement) or too large, are refused before any device call."""
    c = ctypes.c_void_p()
    assert L.aao_create_2d(*args, ctypes.byref(c)) == code
    assert not c.value


def test_create_rejects_null_out(L):
    assert L.aao_create(4, 4, 0.1, 0, None) == -1


def test_null_context_is_an_argument_error(L):
    assert L.aao_destroy(None) == 0
    assert L.aao_set_kappa(None, 1.0) == -1
    assert L.aao_apply_A(None, None, None, 0) == -1
    assert L.aao_gmres(None, None, None, 30, 1e-8, 10, None) == -1


def test_status_strings(L):
    for st, txt in [(0, b"ok"), (1, b"not converged"), (-1, b"invalid argument"),
                    (-4, b"numerical breakdown")]:
        assert L.aao_status_string(st) == txt


def test_oracle_never_imported_by_the_product():
    import subprocess
    import sys
    code = ("import sys, paper_1810_00615_amd, paper_1810_00615_amd.api; "
            "print('oracle' in sys.modules)")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert out.stdout.strip() == "False", out.stdout + out.stderr
