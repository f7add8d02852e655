"""FP64 CPU oracle (test infrastructure only).

Plain, slow, obviously-correct reference for the GPU library: block
Cholesky direct solve, the paper's preconditioner (closed form at the optimal
weights and the definition-based form for any weights), textbook PCG and the
adjoint gradient. The arithmetic lives in ``oracle.c`` (plain C, double
precision); this module only marshals numpy arrays through ctypes.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. The GPU library never does, and the oracle shares no code
with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PC_OPT, PC_SPLIT, PC_NONE = 0, 1, 2
OK, NOT_CONVERGED, EINVAL, ENOTSPD, EBREAKDOWN = 0, 1, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, portable -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_native(dest_dir: str) -> str:
    """Compile oracle.c with -O3 -march=native into ``dest_dir`` (for timing
    the oracle on the host it runs on; the in-tree build stays portable)."""
    out = os.path.join(dest_dir, "liboracle_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c99", "-fPIC",
                           "-shared", "-o", out, _SRC, "-lm"])
    return out


_lib = None


def _bind(path):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    Dd = ctypes.c_double
    sig = {
        "or_spmv": (None, [I, I, P, P, P, P]),
        "or_btchol": (I, [I, I, P, P, P, P]),
        "or_btchol_factor": (I, [I, I, P, P, P, P]),
        "or_btchol_solve": (None, [I, I, P, P, P, P]),
        "or_setup_opt": (I, [I, I, P, P, P, P, P, P, P]),
        "or_apply_Gopt": (None, [I, I, P, P, P, P]),
        "or_apply_Hopt": (None, [I, I, P, P, P, P, P]),
        "or_apply_Gab": (I, [I, I, Dd, Dd, P, P, P, P]),
        "or_apply_Hab": (I, [I, I, Dd, Dd, P, P, P, P]),
        "or_precond": (I, [I, I, I, Dd, Dd, I, P, P, P, P, P]),
        "or_pcg": (I, [I, I, P, P, P, I, Dd, Dd, I, P, Dd, I, P, P, P, P]),
        "or_adjoint": (I, [I, I, P, P, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _bind(_LIB)
    return _lib


class use_library:
    """Context manager: route every call to another build of oracle.c
    (the mutation tests load deliberately broken copies through this)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = _bind(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _dims(D):
    D = np.asarray(D)
    return int(D.shape[0]), int(D.shape[1])


# ---------------------------------------------------------------- matrix A
def spmv(D, O, x):
    """y = A x for the block-tridiagonal A of eq. (1)."""
    N, n = _dims(D)
    D, O, x = _c(D), _c(O), _c(x).reshape(N, n)
    y = np.empty((N, n))
    _load().or_spmv(N, n, _p(D), _p(O), _p(x), _p(y))
    return y


# ---------------------------------------------------------- direct solver
def btchol_solve(D, O, b):
    """x = A^{-1} b by block Cholesky (block Thomas), Section IV-C.

    ``b`` may be (N, n) or (N, n, nrhs). Raises on a non-SPD A.
    """
    N, n = _dims(D)
    D, O = _c(D), _c(O)
    b = np.asarray(b, dtype=np.float64)
    lib = _load()
    Lf = np.empty((N, n, n))
    W = np.empty((max(N - 1, 1), n, n))
    rc = lib.or_btchol_factor(N, n, _p(D), _p(O), _p(Lf), _p(W))
    if rc:
        raise np.linalg.LinAlgError(
            f"A is not SPD (Schur block {-rc - 1} failed)")
    if b.ndim == 3:
        out = np.empty_like(b)
        for j in range(b.shape[2]):
            bj = np.ascontiguousarray(b[:, :, j])
            xj = np.empty((N, n))
            lib.or_btchol_solve(N, n, _p(Lf), _p(W), _p(bj), _p(xj))
            out[:, :, j] = xj
        return out
    bb = _c(b).reshape(N, n)
    x = np.empty((N, n))
    lib.or_btchol_solve(N, n, _p(Lf), _p(W), _p(bb), _p(x))
    return x


# ------------------------------------------------------- preconditioner
def setup_opt(D, O):
    """Closed-form blocks of (G_opt, H_opt), Section IV-A.

    Returns dict(Dinv (N), E (N-1), Hd (N), Hu (N-2), Hl (N-2)); Hu[k] is
    block (k, k+2) and Hl[k] is block (k+2, k) of H_opt.
    """
    N, n = _dims(D)
    D, O = _c(D), _c(O)
    Dinv = np.empty((N, n, n))
    E = np.empty((max(N - 1, 1), n, n))
    Hd = np.empty((N, n, n))
    Hu = np.empty((max(N - 2, 1), n, n))
    Hl = np.empty((max(N - 2, 1), n, n))
    rc = _load().or_setup_opt(N, n, _p(D), _p(O), _p(Dinv), _p(E), _p(Hd),
                              _p(Hu), _p(Hl))
    if rc:
        raise np.linalg.LinAlgError(f"D_{-rc - 1} is not SPD")
    return dict(Dinv=Dinv, E=E[:max(N - 1, 0)], Hd=Hd, Hu=Hu[:max(N - 2, 0)],
                Hl=Hl[:max(N - 2, 0)])


def apply_Gopt(blocks, r):
    N, n = blocks["Dinv"].shape[:2]
    E = blocks["E"] if len(blocks["E"]) else np.zeros((1, n, n))
    y = np.empty((N, n))
    _load().or_apply_Gopt(N, n, _p(_c(blocks["Dinv"])), _p(_c(E)),
                          _p(_c(r).reshape(N, n)), _p(y))
    return y


def apply_Hopt(blocks, v):
    N, n = blocks["Dinv"].shape[:2]
    z = np.zeros((1, n, n))
    Hu = blocks["Hu"] if len(blocks["Hu"]) else z
    Hl = blocks["Hl"] if len(blocks["Hl"]) else z
    y = np.empty((N, n))
    _load().or_apply_Hopt(N, n, _p(_c(blocks["Hd"])), _p(_c(Hu)), _p(_c(Hl)),
                          _p(_c(v).reshape(N, n)), _p(y))
    return y


def apply_Gab(D, O, a, b, r):
    """G_ab r from the splitting definitions (eq. def-GH-ab-multi-splitting)."""
    N, n = _dims(D)
    y = np.empty((N, n))
    rc = _load().or_apply_Gab(N, n, float(a), float(b), _p(_c(D)), _p(_c(O)),
                              _p(_c(r).reshape(N, n)), _p(y))
    if rc:
        raise np.linalg.LinAlgError("D not SPD")
    return y


def apply_Hab(D, O, a, b, v):
    """H_ab v from the splitting definitions (eq. def-GH-ab-multi-splitting)."""
    N, n = _dims(D)
    y = np.empty((N, n))
    rc = _load().or_apply_Hab(N, n, float(a), float(b), _p(_c(D)), _p(_c(O)),
                              _p(_c(v).reshape(N, n)), _p(y))
    if rc:
        raise np.linalg.LinAlgError("D not SPD")
    return y


def _alpha_arr(m, alpha):
    arr = np.ones(16)
    if alpha is not None:
        al = list(alpha)
        for i in range(1, min(m, len(al))):
            arr[i] = float(al[i])
    return arr


def precond(D, O, r, kind=PC_OPT, a=1.0, b=-1.0, m=1, alpha=None):
    """z = M^{-1} r with M^{-1} = (I + a1 H + ... + a_{m-1} H^{m-1}) G.

    ``alpha`` is indexed like the paper: alpha[i] multiplies H^i; alpha[0]
    is ignored (fixed at 1). ``kind``: PC_OPT (closed form at (1,-1)),
    PC_SPLIT (any (a,b) through the splittings), PC_NONE (z = r).
    """
    N, n = _dims(D)
    z = np.empty((N, n))
    al = _alpha_arr(m, alpha)
    rc = _load().or_precond(int(kind), N, n, float(a), float(b), int(m),
                            _p(al), _p(_c(D)), _p(_c(O)),
                            _p(_c(r).reshape(N, n)), _p(z))
    if rc:
        raise np.linalg.LinAlgError("D not SPD")
    return z


def polycoeff(m):
    """The paper's "PolyCoeff" coefficients (Section V footnote):
    alpha_{m-1} = 7 and every other alpha_i = 1; none for m = 1."""
    al = [1.0] * max(m, 1)
    if m > 1:
        al[m - 1] = 7.0
    return al


def pcg(D, O, bvec, kind=PC_OPT, a=1.0, b=-1.0, m=2, alpha=None,
        tol=1e-10, maxit=None, history=False, x0=None):
    """Textbook PCG from x0 = 0 (or the initial guess ``x0``) with the
    preconditioner of ``precond``; the test is ||r_j|| <= tol ||b||.

    Returns (x, info) with info = dict(status, iters, relres, ratio_last,
    ratio_prev[, hist]); ratio_* = ||r_j|| / (tol ||b||) at the last two
    iterates (the margin of the stopping test).
    """
    N, n = _dims(D)
    if maxit is None:
        maxit = 10 * N * n
    x = np.empty((N, n))
    out = np.zeros(4)
    hist = np.zeros(maxit + 1) if history else None
    al = _alpha_arr(m, alpha)
    st = _load().or_pcg(N, n, _p(_c(D)), _p(_c(O)),
                        _p(_c(bvec).reshape(N, n)), int(kind), float(a),
                        float(b), int(m), _p(al), float(tol), int(maxit),
                        _p(x), _p(out), _p(hist) if history else None,
                        _p(_c(x0).reshape(N, n)) if x0 is not None else None)
    info = dict(status=int(st), iters=int(out[0]), relres=float(out[1]),
                ratio_last=float(out[2]), ratio_prev=float(out[3]))
    if history:
        info["hist"] = hist[:info["iters"] + 1].copy()
    return x, info


def adjoint(D, O, x, g):
    """(lambda, dD, dO) for x = A^{-1} b and upstream gradient g = dL/dx."""
    N, n = _dims(D)
    lam = np.empty((N, n))
    dD = np.empty((N, n, n))
    dO = np.empty((max(N - 1, 1), n, n))
    rc = _load().or_adjoint(N, n, _p(_c(D)), _p(_c(O)),
                            _p(_c(x).reshape(N, n)),
                            _p(_c(g).reshape(N, n)), _p(lam), _p(dD), _p(dO))
    if rc:
        raise np.linalg.LinAlgError("A not SPD")
    return lam, dD, dO[:max(N - 1, 0)]


# ------------------------------------------------ paper's cost accounting
def gemv_per_iteration(kind=PC_OPT, a=1.0, m=2):
    """g_a(m) of Section IV-B: block gemvs per PCG iteration (A p and M^{-1} r).

    2m+2 for a = 0, 5m+1 for a in (0,1), 3m+3 for a = 1. For no
    preconditioner (not covered by the paper) the count is the 3 of A p.
    """
    if kind == PC_NONE:
        return 3
    if a == 0.0:
        return 2 * m + 2
    if a == 1.0:
        return 3 * m + 3
    return 5 * m + 1


def distinct_eigenvalue_bound(N, n, a):
    """d_{Nna} of eq. (distinct-eigenvalues-count)."""
    if a == 1.0:
        return (N // 2) * n if N % 2 == 0 else (N // 2) * n + 1
    return N * n if N % 2 == 0 else 2 * (N // 2) * n + 1


# ----------------------------------------------------------- batches
def batch_slices(offsets):
    """Yield (i, row slice, upper-block slice) of instance i in a batch."""
    offsets = np.asarray(offsets)
    for i in range(len(offsets) - 1):
        r0, r1 = int(offsets[i]), int(offsets[i + 1])
        yield i, slice(r0, r1), slice(r0 - i, r1 - i - 1)
