"""Seeded synthetic inputs: random LQR problems turned into SPD block-tridiagonal
Schur complements.

This module is shared by the CPU oracle, the tests and the benchmark. It holds
no arithmetic of the solver or of its preconditioner: it only draws random
dynamics and costs and forms the matrix of the linear system, the way the
paper's experiments build theirs (Section V: the LQR problem written as a QP,
its KKT system, and the Schur complement with respect to the Hessian).

Problem (states x_0..x_{N-1} in R^nx, controls u_0..u_{N-2} in R^nu):
    min  1/2 sum_k x_k' Q_k x_k + 1/2 sum_k u_k' R_k u_k
    s.t. x_0 = given,  x_{k+1} = A_k x_k + B_k u_k.
With the equality-constraint Jacobian C and the Hessian H = blkdiag(Q, R),
the Schur complement S = C H^-1 C' is block tridiagonal with N diagonal blocks
(block size n = nx):
    D_0 = Q_0^-1
    D_k = Q_k^-1 + A_{k-1} Q_{k-1}^-1 A_{k-1}' + B_{k-1} R_{k-1}^-1 B_{k-1}'
    S_{k+1,k} = -A_k Q_k^-1                (sub-diagonal block)
so the upper block of eq. (1), O_k = S_{k,k+1}, is (-A_k Q_k^-1)' = -Q_k^-1 A_k'.

Distributions: A_k = I + s G_k with G_k i.i.d. N(0,1) (s = 0.1, or 0.05 for
the n = 48 workload), B_k i.i.d. N(0,1), Q_k = diag U[1,10],
R_k = diag U[0.1,1], right-hand sides and targets i.i.d. N(0,1).

Random stream: instance j of a workload with seed ``seed`` draws from
numpy.random.default_rng(SeedSequence([seed, j])) in this order: for each
k = 0..N-2 the pair (G_k, B_k); then the Q diagonals (N x nx); then the R
diagonals ((N-1) x nu); then the right-hand sides; then the targets.
Horizon lengths of a ragged batch come from SeedSequence([seed, 2**31 - 1]).
"""
from __future__ import annotations

import numpy as np

__all__ = ["lqr_instance", "lqr_batch", "WORKLOADS", "workload_seed",
           "kkt_dense"]

_HORIZON_STREAM = 2**31 - 1


def workload_seed(index: int) -> int:
    """Base seed of the i-th standard workload (see ``WORKLOADS``)."""
    return 20250319 + int(index)


# The five standard workloads. Shapes and value distributions follow the
# paper's experiment setting (random LQR Schur complements) at the sizes the
# GPU path is measured on.
WORKLOADS = {
    "single_n6": dict(index=0, B=1, N=32, nx=6, nu=3, s=0.1, nrhs=1,
                      record="f64"),
    "single_n12": dict(index=1, B=1, N=512, nx=12, nu=4, s=0.1, nrhs=1,
                       record="f64"),
    "batch_ragged_n12": dict(index=2, B=2048, N=(16, 256), nx=12, nu=4,
                             s=0.1, nrhs=1, record="f32"),
    "batch_grad_n24": dict(index=3, B=256, N=128, nx=24, nu=8, s=0.1,
                           nrhs=1, record="f32"),
    "multirhs_n48": dict(index=4, B=1, N=4096, nx=48, nu=16, s=0.05,
                         nrhs=64, record="f32"),
}


def lqr_instance(N: int, nx: int, nu: int, seed: int, instance: int = 0,
                 s: float = 0.1, nrhs: int = 1, with_target: bool = False,
                 keep_dynamics: bool = False):
    """Draw one LQR problem and return its block-tridiagonal Schur complement.

    Returns a dict with
      D : (N, nx, nx) float64, diagonal blocks (symmetric)
      O : (N-1, nx, nx) float64, upper blocks O_k = S[k, k+1]
      b : (N, nx) float64 if nrhs == 1 else (N, nx, nrhs)
      t : like b (only with ``with_target``), regression targets
      A, Bm, q, r : the raw dynamics and cost diagonals (``keep_dynamics``)
    """
    if N < 1 or nx < 1 or nu < 0:
        raise ValueError("need N >= 1, nx >= 1, nu >= 0")
    rng = np.random.default_rng(np.random.SeedSequence([int(seed),
                                                        int(instance)]))
    A = np.empty((max(N - 1, 0), nx, nx))
    Bm = np.empty((max(N - 1, 0), nx, nu))
    eye = np.eye(nx)
    for k in range(N - 1):
        A[k] = eye + s * rng.standard_normal((nx, nx))
        Bm[k] = rng.standard_normal((nx, nu))
    q = rng.uniform(1.0, 10.0, size=(N, nx))
    r = rng.uniform(0.1, 1.0, size=(max(N - 1, 0), nu))
    bshape = (N, nx) if nrhs == 1 else (N, nx, nrhs)
    b = rng.standard_normal(bshape)
    t = rng.standard_normal(bshape) if with_target else None

    qi = 1.0 / q                       # diagonals of Q_k^-1
    ri = 1.0 / r                       # diagonals of R_k^-1
    D = np.zeros((N, nx, nx))
    D[:, np.arange(nx), np.arange(nx)] = qi
    if N > 1:
        AQ = A * qi[:-1, None, :]      # A_k Q_k^-1
        BR = Bm * ri[:, None, :]       # B_k R_k^-1
        D[1:] += np.einsum("kij,klj->kil", AQ, A)
        D[1:] += np.einsum("kij,klj->kil", BR, Bm)
        O = -np.transpose(AQ, (0, 2, 1)).copy()   # -(A_k Q_k^-1)'
    else:
        O = np.zeros((0, nx, nx))
    D = 0.5 * (D + np.transpose(D, (0, 2, 1)))  # exact symmetry
    out = dict(D=D, O=O, b=b)
    if with_target:
        out["t"] = t
    if keep_dynamics:
        out.update(A=A, Bm=Bm, q=q, r=r)
    return out


def lqr_batch(B: int, N, nx: int, nu: int, seed: int, s: float = 0.1,
              with_target: bool = False, record: str = "f64"):
    """Draw a batch of independent LQR instances, rows concatenated.

    ``N`` is an int (equal horizons) or a pair (lo, hi) for horizons drawn
    uniformly from {lo..hi}. ``record`` = "f32" rounds D and O to float32
    (the system of record of the single-precision workloads; every consumer
    promotes these values exactly).

    Returns dict(D (R,n,n), O (R-B,n,n), b (R,n), offsets (B+1,) int64,
    horizons (B,) int64[, t]) where R = sum of horizons and instance i owns
    rows offsets[i]..offsets[i+1]-1 and upper blocks
    offsets[i]-i .. offsets[i+1]-i-2.
    """
    if isinstance(N, (tuple, list)):
        lo, hi = int(N[0]), int(N[1])
        hr = np.random.default_rng(np.random.SeedSequence([int(seed),
                                                           _HORIZON_STREAM]))
        horizons = hr.integers(lo, hi + 1, size=B).astype(np.int64)
    else:
        horizons = np.full(B, int(N), dtype=np.int64)
    offsets = np.zeros(B + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(horizons)
    R = int(offsets[-1])
    D = np.empty((R, nx, nx))
    O = np.empty((R - B, nx, nx))
    b = np.empty((R, nx))
    t = np.empty((R, nx)) if with_target else None
    for i in range(B):
        inst = lqr_instance(int(horizons[i]), nx, nu, seed, i, s=s,
                            with_target=with_target)
        r0, r1 = offsets[i], offsets[i + 1]
        D[r0:r1] = inst["D"]
        O[r0 - i:r1 - i - 1] = inst["O"]
        b[r0:r1] = inst["b"]
        if with_target:
            t[r0:r1] = inst["t"]
    if record == "f32":
        D = D.astype(np.float32).astype(np.float64)
        O = O.astype(np.float32).astype(np.float64)
    elif record != "f64":
        raise ValueError("record must be 'f64' or 'f32'")
    out = dict(D=D, O=O, b=b, offsets=offsets, horizons=horizons)
    if with_target:
        out["t"] = t
    return out


def kkt_dense(A, Bm, q, r):
    """Dense pieces of the LQR QP: equality Jacobian C and Hessian H.

    Decision vector z = (x_0, u_0, x_1, u_1, ..., u_{N-2}, x_{N-1}).
    Constraint rows: x_0 = given, then x_{k+1} - A_k x_k - B_k u_k = 0.
    Used only by tests, to check that the block Schur complement built by
    ``lqr_instance`` equals C H^-1 C'.
    """
    N = q.shape[0]
    nx = q.shape[1]
    nu = r.shape[1] if r.ndim == 2 and r.shape[0] > 0 else 0
    nz = N * nx + (N - 1) * nu
    xo = lambda k: k * (nx + nu)           # offset of x_k in z
    uo = lambda k: k * (nx + nu) + nx      # offset of u_k in z
    H = np.zeros((nz, nz))
    for k in range(N):
        H[xo(k):xo(k) + nx, xo(k):xo(k) + nx] = np.diag(q[k])
    for k in range(N - 1):
        H[uo(k):uo(k) + nu, uo(k):uo(k) + nu] = np.diag(r[k])
    C = np.zeros((N * nx, nz))
    C[0:nx, xo(0):xo(0) + nx] = np.eye(nx)
    for k in range(N - 1):
        rows = slice((k + 1) * nx, (k + 2) * nx)
        C[rows, xo(k + 1):xo(k + 1) + nx] = np.eye(nx)
        C[rows, xo(k):xo(k) + nx] = -A[k]
        C[rows, uo(k):uo(k) + nu] = -Bm[k]
    return C, H
