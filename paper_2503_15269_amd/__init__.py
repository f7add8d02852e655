"""btpcg: PCG with the multi-splitting polynomial preconditioner of
Yang, Ohtsuka, Plancher and Jones (arXiv 2503.15269) on MI355X.

Thin Python binding of the C-ABI library ``libbtpcg.so`` (declared in
``include/btpcg.h``). This module only marshals arguments: every step of the
solver runs in the library's HIP kernels. PyTorch supplies device memory and
streams. There is no CPU fallback: without the built library, or without a
GPU, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbtpcg.so")

OK, NOT_CONVERGED, EINVAL, ENOTSPD, EBREAKDOWN, ENONFINITE, EHIP, ENOSPACE = \
    0, 1, -1, -2, -3, -4, -5, -6
ETIMEOUT = -7
ESTAGNATED = -8
F64, F32, F32_IR, BF16X2_IR = 0, 1, 2, 3
DT_F64, DT_F32 = 0, 1
PC_POLY, PC_NONE = 0, 1
MAX_M = 8

INFO_DTYPE = np.dtype([("status", "<i4"), ("iters", "<i4"), ("outer", "<i4"),
                       ("fail_index", "<i4"), ("relres", "<f8"),
                       ("relres_true", "<f8"), ("gemv_exec", "<i8"),
                       ("gemv_paper", "<i8")])


class _Params(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double),
                ("m", ctypes.c_int), ("pc", ctypes.c_int),
                ("alpha", ctypes.c_double * MAX_M), ("prec", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("warm_start", ctypes.c_int), ("fallback_f64", ctypes.c_int)]


class BtError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbtpcg.so and declare its C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with "
            "`python -m paper_2503_15269_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    P, I, Dd, Sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    PP = ctypes.POINTER(ctypes.c_void_p)
    PPar = ctypes.POINTER(_Params)
    sig = {
        "bt_default_params": (None, [PPar]),
        "bt_strerror": (ctypes.c_char_p, [I]),
        "bt_workspace_bytes": (Sz, [I, P, I, PPar]),
        "bt_batch_setup": (I, [PP, I, P, I, I, P, P, PPar, P, Sz, P]),
        "bt_setup": (I, [PP, I, I, I, P, P, PPar, P, Sz, P]),
        "bt_refactor": (I, [P, P]),
        "bt_precondition": (I, [P, P, P, P]),
        "bt_solve": (I, [P, P, P, Dd, I, P, P]),
        "bt_solve_batched": (I, [P, P, P, Dd, I, P, P]),
        "bt_solve_adjoint": (I, [P, P, P, P, P, P, Dd, I, P, P]),
        "bt_mrhs_workspace_bytes": (Sz, [P, I]),
        "bt_direct_workspace_bytes": (Sz, [P]),
        "bt_solve_direct": (I, [P, P, P, P, P, Sz, P]),
        "bt_solve_mrhs": (I, [P, I, P, P, Dd, I, P, P, Sz, P]),
        "bt_grid_workspace_bytes": (Sz, [P]),
        "bt_solve_grid": (I, [P, P, P, Dd, I, P, P, Sz, P]),
        "bt_solve_grid_noalloc": (I, [P, P, P, Dd, I, P, P]),
        "bt_set_grid_wait": (I, [P, Dd]),
        "bt_kernel_config_count": (I, []),
        "bt_kernel_config": (I, [I, ctypes.POINTER(I), ctypes.POINTER(I),
                                 ctypes.POINTER(I)]),
        "bt_set_kernel_config": (I, [P, I]),
        "bt_get_kernel_config": (I, [P]),
        "bt_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names the C-ABI exports (every function of include/btpcg.h)."""
    return ["bt_default_params", "bt_strerror", "bt_workspace_bytes",
            "bt_batch_setup", "bt_setup", "bt_refactor", "bt_precondition",
            "bt_solve", "bt_solve_batched", "bt_solve_adjoint",
            "bt_mrhs_workspace_bytes", "bt_solve_mrhs",
            "bt_direct_workspace_bytes", "bt_solve_direct",
            "bt_grid_workspace_bytes", "bt_solve_grid",
            "bt_solve_grid_noalloc", "bt_set_grid_wait",
            "bt_kernel_config_count", "bt_kernel_config",
            "bt_set_kernel_config", "bt_get_kernel_config", "bt_destroy"]


def strerror(code: int) -> str:
    return load_library().bt_strerror(int(code)).decode()


def polycoeff(m: int):
    """The paper's "PolyCoeff" coefficients (Section V): alpha_{m-1} = 7,
    the other alpha_i = 1."""
    al = [1.0] * max(m, 1)
    if m > 1:
        al[m - 1] = 7.0
    return al


@dataclass
class Params:
    """Preconditioner and precision (mirrors ``bt_params``).

    a, b: splitting weights on 2a+b = 1, a >= 0, b >= -1 (b defaults to
    1-2a); m: polynomial order; alpha[i] multiplies H^i (alpha[0] ignored;
    default: all ones); pc: "poly" or "none"; prec: "f64", "f32", "f32_ir";
    warm_start: the solves start from the x passed in (initial guess)
    instead of 0.
    fallback_f64: under "f32_ir", a system whose refinement stagnates is
    finished in float64 on the device (the workspace holds float64 factors
    too); without it such a system stops with status ESTAGNATED.
    """
    a: float = 1.0
    b: Optional[float] = None
    m: int = 2
    alpha: Optional[Sequence[float]] = None
    pc: str = "poly"
    prec: str = "f64"
    max_outer: int = 30
    inner_tol: float = 1e-4
    warm_start: bool = False
    fallback_f64: bool = False

    @staticmethod
    def polycoeff(m: int = 2, **kw) -> "Params":
        return Params(a=1.0, m=m, alpha=polycoeff(m), **kw)

    @staticmethod
    def block_jacobi(m: int = 1, **kw) -> "Params":
        return Params(a=0.0, m=m, **kw)

    def to_c(self) -> _Params:
        p = _Params()
        load_library().bt_default_params(ctypes.byref(p))
        p.a = float(self.a)
        p.b = float(1.0 - 2.0 * self.a if self.b is None else self.b)
        p.m = int(self.m)
        al = [1.0] * MAX_M
        if self.alpha is not None:
            for i, v in enumerate(list(self.alpha)[:MAX_M]):
                al[i] = float(v)
        for i in range(MAX_M):
            p.alpha[i] = al[i]
        p.pc = {"poly": PC_POLY, "none": PC_NONE}[self.pc]
        p.prec = {"f64": F64, "f32": F32, "f32_ir": F32_IR,
                  "bf16x2_ir": BF16X2_IR}[self.prec]
        p.max_outer = int(self.max_outer)
        p.inner_tol = float(self.inner_tol)
        p.warm_start = 1 if self.warm_start else 0
        p.fallback_f64 = 1 if self.fallback_f64 else 0
        return p


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("btpcg needs a ROCm GPU (torch.cuda is unavailable)")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc, what):
    if rc != OK:
        raise BtError(rc, what)


def kernel_configs():
    """[(index, threads, elements_per_thread, prec)] of the solve kernel."""
    lib = load_library()
    out = []
    for i in range(lib.bt_kernel_config_count()):
        nt, s, pr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.bt_kernel_config(i, ctypes.byref(nt), ctypes.byref(s),
                                    ctypes.byref(pr)), "bt_kernel_config")
        out.append((i, nt.value, s.value, pr.value))
    return out


def infos_to_numpy(info_tensor):
    """Device bt_info array -> numpy structured array (synchronises)."""
    raw = info_tensor.detach().cpu().numpy().tobytes()
    return np.frombuffer(raw, dtype=INFO_DTYPE).copy()


def check_infos(info_tensor, what="solve"):
    """Raise BtError on the first instance whose status is not OK
    (synchronises); returns the infos as a numpy structured array."""
    inf = infos_to_numpy(info_tensor)
    bad = np.nonzero(inf["status"] != OK)[0]
    if len(bad):
        i = int(bad[0])
        raise BtError(int(inf["status"][i]),
                      f"{what}: instance {i} of {len(inf)} "
                      f"({len(bad)} not converged)")
    return inf


class Handle:
    """A set-up batch of SPD block-tridiagonal systems (``bt_batch_setup``).

    D: cuda tensor [R, n, n] (float64 or float32 record); O: [R-B, n, n],
    same dtype; offsets: host sequence of B+1 row offsets (None: one system).
    The tensors are referenced, not copied: keep them unchanged (or call
    ``refactor`` after changing them in place).
    """

    def __init__(self, D, O, offsets=None, params: Optional[Params] = None,
                 stream=None):
        torch = _torch()
        lib = load_library()
        self.params = params or Params.polycoeff(2)
        if D.dim() != 3 or D.shape[1] != D.shape[2]:
            raise ValueError("D must be [R, n, n]")
        if not D.is_cuda or not D.is_contiguous():
            raise ValueError("D must be a contiguous cuda tensor")
        R, n = int(D.shape[0]), int(D.shape[1])
        if offsets is None:
            offsets = [0, R]
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        B = len(off) - 1
        if O is None or O.numel() == 0:
            O = None
        else:
            if O.dtype != D.dtype or not O.is_cuda or not O.is_contiguous():
                raise ValueError("O must be a contiguous cuda tensor like D")
            if tuple(O.shape) != (R - B, n, n):
                raise ValueError(f"O must be [{R - B}, {n}, {n}]")
        if D.dtype == torch.float64:
            dtype = DT_F64
        elif D.dtype == torch.float32:
            dtype = DT_F32
        else:
            raise ValueError("D must be float64 or float32")
        self._cp = self.params.to_c()
        ws = lib.bt_workspace_bytes(B, off.ctypes.data_as(ctypes.c_void_p), n,
                                    ctypes.byref(self._cp))
        if ws == 0:
            raise BtError(EINVAL, "bt_workspace_bytes")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=D.device)
        self.D, self.O, self.offsets = D, O, off
        self.B, self.R, self.n = B, R, n
        self.device = D.device
        h = ctypes.c_void_p()
        rc = lib.bt_batch_setup(ctypes.byref(h), B,
                                off.ctypes.data_as(ctypes.c_void_p), n, dtype,
                                _ptr(D), _ptr(O) if O is not None else None,
                                ctypes.byref(self._cp), _ptr(self.workspace),
                                ws, _stream(torch, stream))
        _check(rc, "bt_batch_setup")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.bt_destroy(h)
            self._h = None

    # -- configuration -------------------------------------------------
    def set_kernel_config(self, i: int):
        _check(load_library().bt_set_kernel_config(self._h, int(i)),
               "bt_set_kernel_config")

    def kernel_config(self) -> int:
        return load_library().bt_get_kernel_config(self._h)

    def set_grid_wait(self, seconds: float):
        """Longest wait of one grid barrier of solve_grid before the solve
        gives up with status ETIMEOUT (default 2 s)."""
        _check(load_library().bt_set_grid_wait(self._h, float(seconds)),
               "bt_set_grid_wait")

    def refactor(self, stream=None):
        torch = _torch()
        _check(load_library().bt_refactor(self._h, _stream(torch, stream)),
               "bt_refactor")

    # -- calls -----------------------------------------------------------
    def _vec(self, v, name):
        torch = _torch()
        if v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 cuda tensor")
        if v.numel() != self.R * self.n:
            raise ValueError(f"{name} must have {self.R * self.n} entries")
        return v

    def _start(self, x, b):
        """Output buffer; under ``warm_start`` also the initial guess."""
        if x is None:
            if self.params.warm_start:
                raise ValueError("warm_start: pass the initial guess as x")
            return _torch().empty_like(b)
        return self._vec(x, "x")

    def default_maxit(self):
        return 10 * int(np.max(np.diff(self.offsets))) * self.n

    def solve(self, b, tol: float = 1e-10, maxit: Optional[int] = None,
              x=None, info=None, stream=None):
        """x = A^{-1} b for every system; returns (x, info) on the device.
        With ``warm_start`` the iteration starts from the ``x`` passed in."""
        torch = _torch()
        b = self._vec(b, "b")
        x = self._start(x, b)
        if info is None:
            info = torch.empty(self.B * INFO_DTYPE.itemsize, dtype=torch.uint8,
                               device=self.device)
        maxit = self.default_maxit() if maxit is None else int(maxit)
        rc = load_library().bt_solve_batched(self._h, _ptr(b), _ptr(x),
                                             float(tol), maxit, _ptr(info),
                                             _stream(torch, stream))
        _check(rc, "bt_solve_batched")
        return x, info

    def solve_mrhs(self, B, tol: float = 1e-10, maxit: Optional[int] = None,
                   X=None, stream=None):
        """X = A^{-1} B for a panel of right-hand sides B [R, n, nrhs]
        (float64, cuda). Needs prec "bf16x2_ir". Returns (X, info[nrhs])."""
        torch = _torch()
        if B.dim() != 3 or B.shape[0] != self.R or B.shape[1] != self.n:
            raise ValueError("B must be [R, n, nrhs]")
        if B.dtype != torch.float64 or not B.is_contiguous() or not B.is_cuda:
            raise ValueError("B must be a contiguous float64 cuda tensor")
        nrhs = int(B.shape[2])
        lib = load_library()
        nbytes = lib.bt_mrhs_workspace_bytes(self._h, nrhs)
        if nbytes == 0:
            raise BtError(EINVAL, "bt_mrhs_workspace_bytes")
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if X is None:
            if self.params.warm_start:
                raise ValueError("warm_start: pass the initial guess as X")
            X = torch.empty_like(B)
        elif (X.shape != B.shape or X.dtype != torch.float64 or
              not X.is_contiguous() or not X.is_cuda):
            raise ValueError("X must be a contiguous float64 cuda tensor "
                             "shaped like B")
        info = torch.empty(nrhs * INFO_DTYPE.itemsize, dtype=torch.uint8,
                           device=self.device)
        maxit = self.default_maxit() if maxit is None else int(maxit)
        rc = lib.bt_solve_mrhs(self._h, nrhs, _ptr(B), _ptr(X), float(tol),
                               maxit, _ptr(info), _ptr(scratch), nbytes,
                               _stream(torch, stream))
        _check(rc, "bt_solve_mrhs")
        return X, info

    def solve_direct(self, b, x=None, info=None, scratch=None, stream=None):
        """x = A^{-1} b for every system by block Cholesky (float64, no
        preconditioner, no iteration); n in 1..16, 24, 32, 48, 64. Returns
        (x, info)."""
        torch = _torch()
        b = self._vec(b, "b")
        lib = load_library()
        nbytes = lib.bt_direct_workspace_bytes(self._h)
        if nbytes == 0:
            raise BtError(EINVAL, "bt_direct_workspace_bytes")
        if scratch is None:
            scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if x is None:
            x = torch.empty_like(b)
        if info is None:
            info = torch.empty(self.B * INFO_DTYPE.itemsize, dtype=torch.uint8,
                               device=self.device)
        _check(lib.bt_solve_direct(self._h, _ptr(b), _ptr(x), _ptr(info),
                                   _ptr(scratch), scratch.numel(),
                                   _stream(torch, stream)), "bt_solve_direct")
        return x, info

    def solve_grid(self, b, tol=1e-10, maxit=None, x=None, info=None,
                   scratch=None, stream=None):
        """Solve the handle's single system spread over the whole GPU, one
        persistent launch (bt_solve_grid). Returns (x, info)."""
        torch = _torch()
        b = self._vec(b, "b")
        lib = load_library()
        nbytes = lib.bt_grid_workspace_bytes(self._h)
        if nbytes == 0:
            raise BtError(EINVAL, "bt_grid_workspace_bytes")
        if scratch is None:
            scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        x = self._start(x, b)
        if info is None:
            info = torch.empty(INFO_DTYPE.itemsize, dtype=torch.uint8,
                               device=self.device)
        if maxit is None:
            maxit = self.default_maxit()
        _check(lib.bt_solve_grid(self._h, _ptr(b), _ptr(x), float(tol),
                                 int(maxit), _ptr(info), _ptr(scratch),
                                 scratch.numel(), _stream(torch, stream)),
               "bt_solve_grid")
        return x, info

    def solve_grid_noalloc(self, b, tol=1e-10, maxit=None, x=None,
                           info=None, stream=None):
        """bt_solve_grid with the library's own static scratch instead of a
        workspace (bt_solve_grid_noalloc): no device allocation in the
        library. ``x`` and ``info`` may be passed in so that the call
        allocates nothing on the torch side either. Returns (x, info)."""
        torch = _torch()
        b = self._vec(b, "b")
        x = self._start(x, b)
        if info is None:
            info = torch.empty(INFO_DTYPE.itemsize, dtype=torch.uint8,
                               device=self.device)
        if maxit is None:
            maxit = self.default_maxit()
        _check(load_library().bt_solve_grid_noalloc(
            self._h, _ptr(b), _ptr(x), float(tol), int(maxit), _ptr(info),
            _stream(torch, stream)), "bt_solve_grid_noalloc")
        return x, info

    def precondition(self, r, z=None, stream=None):
        torch = _torch()
        r = self._vec(r, "r")
        if z is None:
            z = torch.empty_like(r)
        _check(load_library().bt_precondition(self._h, _ptr(r), _ptr(z),
                                              _stream(torch, stream)),
               "bt_precondition")
        return z

    def adjoint(self, x, g, tol: float = 1e-10, maxit: Optional[int] = None,
                need_dD: bool = True, need_dO: bool = True, stream=None):
        """(lambda, dD, dO, info) for x = A^{-1} b and g = dL/dx."""
        torch = _torch()
        x = self._vec(x, "x")
        g = self._vec(g, "g")
        lam = torch.empty_like(g)
        dD = torch.empty((self.R, self.n, self.n), dtype=torch.float64,
                         device=self.device) if need_dD else None
        dO = torch.empty((self.R - self.B, self.n, self.n),
                         dtype=torch.float64,
                         device=self.device) if need_dO else None
        info = torch.empty(self.B * INFO_DTYPE.itemsize, dtype=torch.uint8,
                           device=self.device)
        maxit = self.default_maxit() if maxit is None else int(maxit)
        rc = load_library().bt_solve_adjoint(
            self._h, _ptr(x), _ptr(g), _ptr(lam), _ptr(dD),
            _ptr(dO) if dO is not None and dO.numel() else None, float(tol),
            maxit, _ptr(info), _stream(torch, stream))
        _check(rc, "bt_solve_adjoint")
        return lam, dD, dO, info


def _autograd():
    import torch

    class BtSolve(torch.autograd.Function):
        """x = A(D, O)^{-1} b with the adjoint backward of the paper's
        preconditioned solve: dL/db = lambda = A^{-1} g,
        dL/dD_k = -lambda_k x_k^T, dL/dO_k = -(lambda_k x_{k+1}^T +
        x_k lambda_{k+1}^T)."""

        @staticmethod
        def forward(ctx, D, O, b, offsets=None, params=None, tol=1e-10,
                    maxit=None, check=True):
            h = Handle(D.detach(), O.detach() if O is not None else None,
                       offsets, params)
            x, info = h.solve(b.detach().reshape(-1).contiguous(), tol, maxit)
            if check:  # a failed solve must not reach autograd silently
                check_infos(info, "BtSolve forward")
            ctx.h, ctx.tol, ctx.maxit, ctx.check = h, tol, maxit, check
            ctx.bshape = b.shape
            ctx.info = info
            ctx.save_for_backward(x)
            return x.view(b.shape)

        @staticmethod
        def backward(ctx, gx):
            (x,) = ctx.saved_tensors
            g = gx.reshape(-1).to(torch.float64).contiguous()
            lam, dD, dO, info = ctx.h.adjoint(x, g, ctx.tol, ctx.maxit,
                                              need_dD=ctx.needs_input_grad[0],
                                              need_dO=ctx.needs_input_grad[1])
            if ctx.check:
                check_infos(info, "BtSolve backward (adjoint)")
            ctx.adj_info = info
            D, O = ctx.h.D, ctx.h.O
            gD = dD.to(D.dtype) if dD is not None else None
            gO = dO.to(O.dtype) if (dO is not None and O is not None) else None
            return gD, gO, lam.view(ctx.bshape), None, None, None, None, None

    return BtSolve


_BtSolve = None


def bt_solve(D, O, b, offsets=None, params=None, tol=1e-10, maxit=None,
             check=True):
    """Differentiable solve (torch.autograd.Function ``BtSolve``). With
    ``check`` (default) the forward and the adjoint raise BtError when an
    instance did not converge (this synchronises; pass False under graph
    capture and read the infos instead)."""
    global _BtSolve
    if _BtSolve is None:
        _BtSolve = _autograd()
    return _BtSolve.apply(D, O, b, offsets, params, tol, maxit, check)


def BtSolve():
    """The torch.autograd.Function class itself."""
    global _BtSolve
    if _BtSolve is None:
        _BtSolve = _autograd()
    return _BtSolve
