"""Python front end of libaao: torch tensors in, torch tensors out.

torch supplies device memory and the stream; every step of the computation runs
in the library's HIP kernels (see include/aao.h).  All vectors are float64 and
contiguous on the problem's device; a vector of the monolithic system is an
(ell, n) tensor whose row k holds time level k+1.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from ._lib import (BATCH_CONFIG_KINDS, CONFIG_KINDS, GMRES_CGS2_CLASSIC, GMRES_EARLY_CHECK, GMRES_TRANSPOSE,
                   GMRES_ZERO_GUESS, KERNELS, AAOError, Info, check, lib)

HEAT, BD2, BD4, CD = 0, 1, 2, 3
SCHEMES = {"heat": HEAT, "heat_ie": HEAT, "bd2": BD2, "wave_bd2": BD2, "bd4": BD4,
           "wave_bd4": BD4, "cd": CD, "wave_cd": CD}
PRECISIONS = {"fp64": 0, "mixed": 1, "fp32": 2, "mixed_in": 3}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _cgs2_flag(cgs2):
    if cgs2 not in ("delayed", "classic"):
        raise ValueError("cgs2 must be 'delayed' or 'classic'")
    return GMRES_CGS2_CLASSIC if cgs2 == "classic" else 0


def set_tune_cache(path: Optional[str]):
    """Process-wide file of tuned launch shapes (aao_set_tune_cache); None = none."""
    st = lib().aao_set_tune_cache(None if path is None else str(path).encode())
    check(st, "aao_set_tune_cache")


def _device(device):
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


class Problem:
    """One all-at-once system A U = b (arXiv 1810.00615, Sec. 2) on one GPU.

    Parameters follow the paper's statement of the problem: n interior nodes,
    ell time steps of size tau (default 1/ell, i.e. T = 1), the scheme
    ("heat" = implicit Euler; for the wave equation "bd2" / "bd4" = two- / four-step
    backward differences, "cd" = central differences), the coefficient kappa of K,
    optional variable steps (heat) and the precision of the preconditioner apply
    ("fp64", "mixed", "fp32", "mixed_in")."""

    def __init__(self, n: int, ell: int, tau: Optional[float] = None, scheme="heat",
                 kappa: float = 1.0, precision: str = "fp64", steps=None, neumann_order: int = 0,
                 device="cuda"):
        self.n = int(n)
        self.ell = int(ell)
        self.tau = float(tau) if tau is not None else 1.0 / self.ell
        self.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        self.device = _device(device)
        if self.device.type != "cuda":
            raise ValueError("the all-at-once library runs on a GPU device only")
        self._L = lib()
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            where, st = self._create()
        check(st, where)
        self.kappa = None
        self.set_kappa(kappa)
        self.precision = None
        self.set_precision(precision)
        self.neumann_order = 0
        self.set_neumann_order(neumann_order)
        self.steps = None
        if steps is not None:
            self.set_steps(steps)

    def _create(self):
        return "aao_create", self._L.aao_create(self.n, self.ell, self.tau, self.scheme,
                                                ctypes.byref(self._ctx))

    # -------------------------------------------------------------- setup
    def _c(self, st, where):
        return check(st, where, self._ctx)

    def close(self):
        if self._ctx:
            self._L.aao_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_kappa(self, kappa: float):
        self._c(self._L.aao_set_kappa(self._ctx, float(kappa)), "aao_set_kappa")
        self.kappa = float(kappa)

    def set_precision(self, precision: str):
        self._c(self._L.aao_set_precision(self._ctx, PRECISIONS[precision]), "aao_set_precision")
        self.precision = precision

    def set_neumann_order(self, q: int):
        self._c(self._L.aao_set_neumann_order(self._ctx, int(q)), "aao_set_neumann_order")
        self.neumann_order = int(q)

    def set_steps(self, steps):
        if steps is None:
            self._c(self._L.aao_set_steps(self._ctx, None), "aao_set_steps")
            self.steps = None
            return
        arr = np.ascontiguousarray(np.asarray(steps, dtype=np.float64))
        if arr.shape != (self.ell,):
            raise ValueError(f"steps must have shape ({self.ell},)")
        self._c(self._L.aao_set_steps(self._ctx, arr.ctypes.data_as(ctypes.c_void_p)),
                "aao_set_steps")
        self.steps = arr

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self._c(self._L.aao_set_stream(self._ctx, ctypes.c_void_p(s)), "aao_set_stream")

    def _vec(self, x: torch.Tensor, shape, name):
        if not isinstance(x, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if x.dtype != torch.float64 or x.device != self.device or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if tuple(x.shape) != tuple(shape) and x.numel() != int(np.prod(shape)):
            raise ValueError(f"{name} must have shape {shape}")
        return x

    def empty(self):
        return torch.empty((self.ell, self.n), dtype=torch.float64, device=self.device)

    def zeros(self):
        return torch.zeros((self.ell, self.n), dtype=torch.float64, device=self.device)

    # ----------------------------------------------------------- operators
    def project_sine(self, modes, amps) -> torch.Tensor:
        """L2 projection onto the P1 space of sum_m amps[m] sin(modes[m] pi x)."""
        modes = np.ascontiguousarray(np.asarray(modes, dtype=np.int32))
        amps = np.ascontiguousarray(np.asarray(amps, dtype=np.float64))
        u0 = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._stream()
        self._c(self._L.aao_project_sine(self._ctx, len(modes), modes.ctypes.data_as(ctypes.c_void_p),
                                         amps.ctypes.data_as(ctypes.c_void_p), _ptr(u0)),
                "aao_project_sine")
        return u0

    def rhs(self, u0: torch.Tensor, v0: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._vec(u0, (self.n,), "u0")
        if v0 is not None:
            self._vec(v0, (self.n,), "v0")
        b = self.empty()
        self._stream()
        self._c(self._L.aao_build_rhs(self._ctx, _ptr(u0), _ptr(v0), _ptr(b)), "aao_build_rhs")
        return b

    def A(self, x: torch.Tensor, transpose: bool = False, out=None) -> torch.Tensor:
        self._vec(x, (self.ell, self.n), "x")
        y = self.empty() if out is None else self._vec(out, (self.ell, self.n), "out")
        self._stream()
        self._c(self._L.aao_apply_A(self._ctx, _ptr(x), _ptr(y), int(transpose)), "aao_apply_A")
        return y

    def Pinv(self, r: torch.Tensor, order: int = 0, transpose: bool = False, out=None):
        self._vec(r, (self.ell, self.n), "r")
        z = self.empty() if out is None else self._vec(out, (self.ell, self.n), "out")
        self._stream()
        self._c(self._L.aao_apply_Pinv(self._ctx, _ptr(r), _ptr(z), int(order), int(transpose)),
                "aao_apply_Pinv")
        return z

    def solve(self, b: torch.Tensor, restart: int = 30, tol: float = 1e-8, maxit: int = 300,
              x0: Optional[torch.Tensor] = None, out=None, cgs2: str = "delayed",
              early_check: bool = False):
        """FGMRES(restart) with the circulant preconditioner; returns (U, info).
        cgs2: "delayed" (re-orthogonalisation deferred by one step) or "classic"
        (three passes); early_check: check the column before the update pass at every
        step (AAO_GMRES_EARLY_CHECK)."""
        self._vec(b, (self.ell, self.n), "b")
        x = out if out is not None else self.empty()
        flags = _cgs2_flag(cgs2) | (GMRES_EARLY_CHECK if early_check else 0)
        if x0 is None:
            flags |= GMRES_ZERO_GUESS
        else:
            x.copy_(x0)
        info = Info()
        self._stream()
        st = self._L.aao_gmres_ex(self._ctx, _ptr(b), _ptr(x), int(restart), float(tol),
                                  int(maxit), flags, ctypes.byref(info))
        self._c(st, "aao_gmres_ex")
        d = info.as_dict()
        d["status"] = st
        return x, d

    def adjoint(self, g: torch.Tensor, restart: int = 30, tol: float = 1e-8, maxit: int = 300,
                out=None):
        """Solve A^T lam = g (preconditioned with C^{-T}); returns (lam, info)."""
        self._vec(g, (self.ell, self.n), "g")
        lam = out if out is not None else self.empty()
        info = Info()
        self._stream()
        st = self._L.aao_gmres_ex(self._ctx, _ptr(g), _ptr(lam), int(restart), float(tol),
                                  int(maxit), GMRES_ZERO_GUESS | GMRES_TRANSPOSE,
                                  ctypes.byref(info))
        self._c(st, "aao_gmres_ex")
        d = info.as_dict()
        d["status"] = st
        return lam, d

    def grad_checkpointed(self, u0, Uck, stride, lam, want_kappa=True, recompute_out=None):
        """(g_u0, g_kappa) from checkpoint rows Uck = U[stride-1::stride] (heat); the
        trajectory between checkpoints is recomputed on the device."""
        gu = torch.empty(self.n, dtype=torch.float64, device=self.device)
        gk = ctypes.c_double(0.0)
        self._stream()
        self._c(self._L.aao_grad_checkpointed(
            self._ctx, _ptr(u0), _ptr(Uck) if Uck is not None and Uck.numel() else None,
            int(stride), _ptr(lam), _ptr(gu), ctypes.byref(gk) if want_kappa else None,
            _ptr(recompute_out)), "aao_grad_checkpointed")
        return gu, (gk.value if want_kappa else None)

    def tune(self, reps: int = 10):
        """Time every admissible launch shape of the forward transform, the shifted
        solves, the inverse transform and the matvec for the current precision mode
        and keep the fastest (aao_tune); returns configs()."""
        self._stream()
        with torch.cuda.device(self.device):
            self._c(self._L.aao_tune(self._ctx, int(reps)), "aao_tune")
        return self.configs()

    def configs(self):
        """{kernel: None (default) or (code, shape)}; shape is (points per thread, W, 0)
        for the transforms, (chunk, threads, staged) for the shifted solves and
        (rows per thread, DPP lane moves, 0) for the matvec."""
        out = {}
        for kind, name in enumerate(CONFIG_KINDS):
            code = ctypes.c_int(0)
            self._c(self._L.aao_get_config(self._ctx, kind, ctypes.byref(code)), "aao_get_config")
            if code.value < 0:
                out[name] = None
                continue
            shape = (ctypes.c_int * 3)()
            self._c(self._L.aao_config_shape(self._ctx, kind, code.value, shape), "aao_config_shape")
            out[name] = (code.value, tuple(shape))
        return out

    def set_config(self, kernel: str, code: int):
        """Pin one kernel's launch shape (code as in configs(); -1 = default)."""
        self._c(self._L.aao_set_config(self._ctx, CONFIG_KINDS.index(kernel), int(code)),
                "aao_set_config")

    def set_timing(self, enable=True):
        """Bracket kernel launches with HIP events (clears the accumulators).  enable:
        True / False for every kernel or none, or an iterable of kernel names."""
        if isinstance(enable, bool) or enable is None:
            mask = (1 << len(KERNELS)) - 1 if enable else 0
        else:
            mask = 0
            for name in enable:
                mask |= 1 << KERNELS.index(name)
        self._c(self._L.aao_set_timing_mask(self._ctx, mask), "aao_set_timing_mask")

    def timing(self):
        """{kernel: (total_ms, launches, algorithmic_bytes)} accumulated since set_timing."""
        out = {}
        for i, name in enumerate(KERNELS):
            t = ctypes.c_double(0.0)
            c = ctypes.c_int64(0)
            b = ctypes.c_double(0.0)
            self._c(self._L.aao_get_timing_ex(self._ctx, i, ctypes.byref(t), ctypes.byref(c),
                                              ctypes.byref(b)), "aao_get_timing_ex")
            out[name] = (t.value, c.value, b.value)
        return out

    def grad(self, U, lam, u0=None, v0=None, want_v0=False):
        """(g_u0, g_v0, g_kappa) of L(U) from the adjoint solution lam."""
        gu = torch.empty(self.n, dtype=torch.float64, device=self.device)
        gv = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_v0 else None
        gk = ctypes.c_double(0.0)
        self._stream()
        self._c(self._L.aao_grad(self._ctx, _ptr(u0), _ptr(v0), _ptr(U), _ptr(lam), _ptr(gu),
                                 _ptr(gv), ctypes.byref(gk)), "aao_grad")
        return gu, gv, gk.value


class Problem2D(Problem):
    """The all-at-once system on the unit square (aao_create_2d): bilinear elements on
    a uniform nx x ny interior grid, M2 = My (x) Mx, K2 = Ky (x) Mx + My (x) Kx, and the
    time structure of `scheme`.  Vectors of the monolithic system are (ell, ny, nx)
    tensors (x fastest); u0 and v0 are (ny, nx).  ny + 1 must be a power of two.
    Variable steps, Neumann terms and the gradient reductions are not available
    here (the adjoint solve is)."""

    def __init__(self, nx: int, ny: int, ell: int, tau: Optional[float] = None,
                 scheme="heat", kappa: float = 1.0, precision: str = "fp64", device="cuda"):
        self.nx = int(nx)
        self.ny = int(ny)
        super().__init__(self.nx * self.ny, ell, tau, scheme, kappa=kappa,
                         precision=precision, device=device)

    def _create(self):
        return "aao_create_2d", self._L.aao_create_2d(self.nx, self.ny, self.ell, self.tau,
                                                      self.scheme, ctypes.byref(self._ctx))

    def empty(self):
        return torch.empty((self.ell, self.ny, self.nx), dtype=torch.float64, device=self.device)

    def zeros(self):
        return torch.zeros((self.ell, self.ny, self.nx), dtype=torch.float64, device=self.device)


__all__ = ["Problem", "Problem2D", "AAOError", "HEAT", "BD2", "set_tune_cache"]


class Batch:
    """Many independent all-at-once problems of uneven size solved together
    (one launch per phase over all problems, hipGraph replay per Arnoldi step).

    A batch vector is a 1-D float64 tensor holding problem p's (ell_p, n_p) array at
    ``offsets[p]``; ``views(vec)`` returns those (ell_p, n_p) views."""

    def __init__(self, ns, ells, kappas, taus=None, scheme="heat", precision="mixed",
                 device="cuda"):
        self.ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int64))
        self.ells = np.ascontiguousarray(np.asarray(ells, dtype=np.int64))
        self.kappas = np.ascontiguousarray(np.asarray(kappas, dtype=np.float64))
        self.taus = None if taus is None else np.ascontiguousarray(np.asarray(taus, dtype=np.float64))
        self.count = len(self.ns)
        self.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        self.device = _device(device)
        self._L = lib()
        self._b = ctypes.c_void_p()
        p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        with torch.cuda.device(self.device):
            st = self._L.aao_batch_create(self.count, p(self.ns), p(self.ells), p(self.taus),
                                          p(self.kappas), self.scheme, PRECISIONS[precision],
                                          ctypes.byref(self._b))
        check(st, "aao_batch_create")
        self.offsets = np.zeros(self.count, dtype=np.int64)
        tot = ctypes.c_int64(0)
        self._c(self._L.aao_batch_offsets(self._b, p(self.offsets), ctypes.byref(tot)),
                "aao_batch_offsets")
        self.total = int(tot.value)
        self.u_offsets = np.concatenate([[0], np.cumsum(self.ns)[:-1]]).astype(np.int64)

    def _c(self, st, where):
        if st < 0:
            detail = self._L.aao_batch_last_error(self._b).decode()
            raise AAOError(st, where, detail)
        return st

    def close(self):
        if self._b:
            self._L.aao_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_in(self):
        # inputs written on torch's stream must land before the batch stream reads them
        torch.cuda.current_stream(self.device).synchronize()

    def empty(self):
        return torch.empty(self.total, dtype=torch.float64, device=self.device)

    def zeros(self):
        return torch.zeros(self.total, dtype=torch.float64, device=self.device)

    def views(self, vec):
        return [vec[o:o + int(n) * int(l)].view(int(l), int(n))
                for o, n, l in zip(self.offsets, self.ns, self.ells)]

    def pack(self, arrays):
        vec = self.zeros()
        for v, a in zip(self.views(vec), arrays):
            v.copy_(torch.as_tensor(a, dtype=torch.float64, device=self.device).view(v.shape))
        return vec

    def set_graph(self, enable: bool):
        self._c(self._L.aao_batch_set_graph(self._b, int(enable)), "aao_batch_set_graph")

    def configs(self):
        """{shape: value} of the batch's launch shapes (aao_batch_get_config)."""
        out = {}
        for kind, name in enumerate(BATCH_CONFIG_KINDS):
            v = ctypes.c_int(0)
            self._c(self._L.aao_batch_get_config(self._b, kind, ctypes.byref(v)),
                    "aao_batch_get_config")
            out[name] = v.value
        return out

    def set_config(self, shape: str, value: int):
        self._c(self._L.aao_batch_set_config(self._b, BATCH_CONFIG_KINDS.index(shape), int(value)),
                "aao_batch_set_config")

    def tune(self, b=None, restart=30, tol=1e-8, maxit=300, reps=3):
        """Time the candidate launch shapes on this batch (with a right-hand side b also
        the graph span, by timing solves of it) and keep the fastest; returns configs()."""
        self._sync_in()
        self._c(self._L.aao_batch_tune(self._b, _ptr(b), int(restart), float(tol), int(maxit),
                                       int(reps)), "aao_batch_tune")
        return self.configs()

    def project_sine(self, modes, amps):
        """u0 for every problem (concatenated n_p-vectors); amps: (count, J)."""
        modes = np.ascontiguousarray(np.asarray(modes, dtype=np.int32))
        amps = np.ascontiguousarray(np.asarray(amps, dtype=np.float64))
        assert amps.shape == (self.count, len(modes))
        u0 = torch.empty(int(self.ns.sum()), dtype=torch.float64, device=self.device)
        self._sync_in()
        self._c(self._L.aao_batch_project_sine(self._b, len(modes),
                                               modes.ctypes.data_as(ctypes.c_void_p),
                                               amps.ctypes.data_as(ctypes.c_void_p), _ptr(u0)),
                "aao_batch_project_sine")
        return u0

    def rhs(self, u0cat):
        b = self.empty()
        self._sync_in()
        self._c(self._L.aao_batch_build_rhs(self._b, _ptr(u0cat), _ptr(b)), "aao_batch_build_rhs")
        return b

    def A(self, x, transpose=False):
        y = self.zeros()
        self._sync_in()
        self._c(self._L.aao_batch_apply_A(self._b, _ptr(x), _ptr(y), int(transpose)),
                "aao_batch_apply_A")
        return y

    def Pinv(self, r, transpose=False):
        z = self.zeros()
        self._sync_in()
        self._c(self._L.aao_batch_apply_Pinv(self._b, _ptr(r), _ptr(z), int(transpose)),
                "aao_batch_apply_Pinv")
        return z

    def solve(self, b, restart=30, tol=1e-8, maxit=300, x0=None, out=None, transpose=False,
              cgs2="delayed"):
        """FGMRES on every problem; x0=None starts from zero (no residual matvec in
        the first cycle; the alignment padding between members of the result is then
        left unwritten); transpose=True solves A_p^T x_p = b_p; cgs2 as in
        Problem.solve."""
        x = out if out is not None else self.empty()
        flags = (GMRES_TRANSPOSE if transpose else 0) | _cgs2_flag(cgs2)
        if x0 is None:
            flags |= GMRES_ZERO_GUESS
        else:
            x.copy_(x0)
        infos = (Info * self.count)()
        self._sync_in()
        st = self._L.aao_batch_gmres_ex(self._b, _ptr(b), _ptr(x), int(restart), float(tol),
                                        int(maxit), flags, ctypes.cast(infos, ctypes.c_void_p))
        self._c(st, "aao_batch_gmres_ex")
        return x, [i.as_dict() for i in infos], st
