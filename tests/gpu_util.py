"""Helpers shared by the GPU tests: seeded inputs -> device tensors -> the HIP
path through the C-ABI binding; oracle references on the CPU."""
import numpy as np

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt


def to_dev(arr, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(arr), dtype=dtype, device="cuda")


def gpu_solve(D, O, b, offsets=None, params=None, tol=1e-10, maxit=None,
              record="f64"):
    """Solve on the GPU; returns (x [R, n] numpy, infos, handle)."""
    import torch
    dt = torch.float64 if record == "f64" else torch.float32
    n = D.shape[1]
    Dt = to_dev(D, dt)
    Ot = to_dev(O, dt) if O is not None and len(O) else None
    bt_ = to_dev(np.asarray(b).reshape(-1), torch.float64)
    h = bt.Handle(Dt, Ot, offsets, params)
    x, info = h.solve(bt_, tol, maxit)
    torch.cuda.synchronize()
    return x.cpu().numpy().reshape(-1, n), bt.infos_to_numpy(info), h


def oracle_kind(params):
    """Map binding parameters to the oracle's preconditioner arguments."""
    if params.pc == "none":
        return dict(kind=orc.PC_NONE)
    a = params.a
    b = 1 - 2 * a if params.b is None else params.b
    kind = orc.PC_OPT if a == 1.0 else orc.PC_SPLIT
    return dict(kind=kind, a=a, b=b, m=params.m, alpha=params.alpha)


def iteration_match(gpu_it, ref_info, margin=1e-6, slack=0):
    """Equal iteration counts, or off by one only when the oracle's stopping
    test was within ``margin`` of its threshold at the last two iterates.
    ``slack`` widens this for runs longer than the dimension of the system
    (plain CG without preconditioner), where CG has lost finite termination
    and the count depends on the rounding order of its dot products."""
    if abs(gpu_it - ref_info["iters"]) <= slack:
        return True
    near = (abs(ref_info["ratio_last"] - 1) < margin or
            abs(ref_info["ratio_prev"] - 1) < margin)
    return near and abs(gpu_it - ref_info["iters"]) == 1


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) /
                 max(np.linalg.norm(np.asarray(b)), 1e-300))


def rowmax_rel(a, b, n=None):
    """Largest error of one block row: ||a_k - b_k|| over the larger of
    ||b_k|| and the root-mean-square block-row norm of b. A wrong block row
    (a short tail, one instance of a batch) shows here even when the global
    relative norm hides it."""
    b = np.asarray(b, dtype=np.float64)
    n = n or b.shape[-1]
    a = np.asarray(a, dtype=np.float64).reshape(-1, n)
    b = b.reshape(-1, n)
    e = np.linalg.norm(a - b, axis=1)
    nb = np.linalg.norm(b, axis=1)
    rms = max(float(np.sqrt(np.mean(nb ** 2))), 1e-300)
    return float(np.max(e / np.maximum(nb, rms)))


def assert_close(a, b, tol, what=""):
    """Global relative error and largest block-row error both within tol."""
    g, r = rel(a, b), rowmax_rel(a, b)
    assert g <= tol and r <= tol, (what, "global", g, "row max", r, "tol", tol)


def true_relres(D, O, b, x):
    """||b - A x|| / ||b|| in float64 with the oracle's product."""
    r = np.asarray(b) - orc.spmv(D, O, np.asarray(x).reshape(np.shape(b)))
    return float(np.linalg.norm(r) / max(np.linalg.norm(b), 1e-300))


# float64 solves stop on the recursive residual at tol; the true residual of
# the returned x may drift above it by rounding: 1 % is allowed
F64_TRUE_RES = 1.01e-10


def workload(name, instances=None):
    """Synthetic inputs of a standard workload (optionally a subset of the
    instances of a batch, drawn with the same per-instance seeds)."""
    w = lqrgen.WORKLOADS[name]
    seed = lqrgen.workload_seed(w["index"])
    if w["B"] == 1:
        d = lqrgen.lqr_instance(w["N"], w["nx"], w["nu"], seed, 0, s=w["s"],
                                nrhs=w["nrhs"],
                                with_target=name == "batch_grad_n24")
        if w["record"] == "f32":
            d["D"] = d["D"].astype(np.float32).astype(np.float64)
            d["O"] = d["O"].astype(np.float32).astype(np.float64)
        return d
    return lqrgen.lqr_batch(w["B"], w["N"], w["nx"], w["nu"], seed, s=w["s"],
                            with_target=name == "batch_grad_n24",
                            record=w["record"])
