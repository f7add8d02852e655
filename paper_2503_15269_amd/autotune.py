"""Autotuner for the batched solve.

Times every applicable solve-kernel configuration (the register-resident
bin kernel and the generic workgroup-size x elements-per-thread variants of
the right precision) and, for float32 iteration with float64 refinement, a
set of inner tolerances, on the caller's own systems. A candidate only
counts if every system converges. The fastest choice is cached per device
and problem signature in a JSON file (``$BTPCG_TUNE_CACHE``, default
``~/.cache/btpcg/autotune.json``).

``tune`` never changes the preconditioner itself (weights, order,
coefficients): it is the method the caller asked for. ``tune_order`` is the
opt-in that also picks the polynomial order m for the caller's systems.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import replace
from typing import Optional, Sequence

import numpy as np

from . import F32, F64, Handle, Params, infos_to_numpy, kernel_configs, OK

INNER_TOLS = (1e-4, 3e-5, 1e-5, 3e-6, 1e-6)
# Candidate inner tolerances of the many-right-hand-side solve: its bfloat16
# split operator is accurate to ~1e-5, so a refinement step gains at most
# ~1e-4..1e-5 whatever the inner solve does; looser inner solves are cheaper.
MRHS_INNER_TOLS = (1e-4, 2e-4, 3e-4, 5e-4)


def _cache_path():
    return os.environ.get("BTPCG_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache",
                                       "btpcg", "autotune.json"))


def _signature(D, offsets, params: Params, tol):
    import torch
    offs = np.asarray(offsets if offsets is not None else [0, D.shape[0]])
    lens = np.diff(offs)
    dev = torch.cuda.get_device_name(D.device)
    return "|".join(str(x) for x in (
        dev, D.shape[1], len(lens), int(lens.max()), int(lens.sum()),
        str(D.dtype), params.prec, params.pc, params.a, params.m,
        tuple(params.alpha or ()), tol))


def _load_cache(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _time(h, b, tol, maxit, reps):
    import torch
    x, info = h.solve(b, tol, maxit)          # warm-up, checks convergence
    torch.cuda.synchronize()
    inf = infos_to_numpy(info)
    if not np.all(inf["status"] == OK):
        return None
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(reps):
        h.refactor()
        ev0.record()
        h.solve(b, tol, maxit, x=x, info=info)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        best = ms if best is None else min(best, ms)
    return best


def tune(D, O, offsets, b, params: Params, tol: float = 1e-10,
         maxit: Optional[int] = None, reps: int = 3,
         inner_tols: Sequence[float] = INNER_TOLS, use_cache: bool = True,
         verbose: bool = False):
    """Return dict(params=Params, kernel_config=int, ms=float, table=[...])."""
    path = _cache_path()
    key = _signature(D, offsets, params, tol)
    cache = _load_cache(path) if use_cache else {}
    if key in cache:
        c = cache[key]
        return dict(params=replace(params, inner_tol=c["inner_tol"]),
                    kernel_config=c["kernel_config"], ms=c["ms"],
                    table=c.get("table", []), cached=True)
    prec = F64 if params.prec == "f64" else F32
    tols = list(inner_tols) if params.prec == "f32_ir" else [params.inner_tol]
    table = []
    best = None
    for t in tols:
        p = replace(params, inner_tol=t)
        h = Handle(D, O, offsets, p)
        cands = [i for i, nt, s, pr in kernel_configs() if pr == prec]
        for cfg in cands:
            try:
                h.set_kernel_config(cfg)
            except RuntimeError:
                continue                      # cannot hold these systems
            ms = _time(h, b, tol, maxit, reps)
            table.append((t, cfg, ms))
            if verbose:
                print(f"autotune inner_tol={t:g} config={cfg}: {ms}")
            if ms is not None and (best is None or ms < best[2]):
                best = (t, cfg, ms)
        del h
    if best is None:
        raise RuntimeError("autotune: no configuration converged")
    res = dict(inner_tol=best[0], kernel_config=best[1], ms=best[2],
               table=table)
    if use_cache:
        cache[key] = res
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, path)
    return dict(params=replace(params, inner_tol=best[0]),
                kernel_config=best[1], ms=best[2], table=table, cached=False)


def tune_order(D, O, offsets, b, params: Params, tol: float = 1e-10,
               orders: Sequence[int] = (1, 2, 3, 4),
               alpha_last: Optional[float] = None, **kw):
    """Also choose the polynomial order m for these systems (an explicit
    opt-in: unlike ``tune`` it changes the preconditioner). Each order runs
    with the caller's weights (a, b) and the "PolyCoeff" coefficients of
    Section V (alpha_{m-1} = ``alpha_last``, default 7, the others 1), and
    goes through ``tune`` (kernel configuration and inner tolerance); the
    fastest order whose every system converges wins.

    Returns ``tune``'s dict for the winner plus ``orders``: {m: ms or None}.
    """
    results, best = {}, None
    for m in orders:
        alpha = [1.0] * m
        if m > 1:
            alpha[m - 1] = 7.0 if alpha_last is None else float(alpha_last)
        p = replace(params, m=int(m), alpha=alpha)
        try:
            r = tune(D, O, offsets, b, p, tol, **kw)
        except RuntimeError:          # no configuration converged
            results[int(m)] = None
            continue
        results[int(m)] = r["ms"]
        if best is None or r["ms"] < best["ms"]:
            best = r
    if best is None:
        raise RuntimeError("autotune: no polynomial order converged")
    best = dict(best)
    best["orders"] = results
    return best
