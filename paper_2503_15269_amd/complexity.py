"""Direct against iterative on the GPU (Section IV-C, eq. complexity-comparison).

The paper argues that block Cholesky costs O(N n^3) whatever the hardware,
because its pivots are sequential along the horizon, while PCG with the
multi-splitting preconditioner costs O(n_itr (N / n_blk)(n^2 / n_thr) g_a(m)
+ (N / n_blk) n^3) when the block rows are spread over n_blk groups of n_thr
threads; so for N >> 1 the iterative method wins. This module measures both
sides of that claim with the library on one GPU, over the horizon N:

* one system: ``bt_solve_direct`` (block Cholesky, float64, the whole
  factorisation and both substitutions, sequential in N) against
  ``bt_refactor`` + PCG (the preconditioner set up over all block rows at
  once, then the iteration), in float64 and in float32 + float64
  refinement; PCG runs on the grid path (``bt_solve_grid``, every step a
  kernel over all block rows) and, where the system fits one workgroup, on
  ``bt_solve`` (the whole iteration inside one workgroup), and the faster
  of the two counts;
* a batch of B systems: the same direct solver, parallel over the batch but
  still sequential in N inside each system, against ``bt_refactor`` +
  ``bt_solve_batched``.

Reported per point: milliseconds of each method (median of a few runs of
the whole call, inputs resident on the device), PCG iterations, the ratio,
and the agreement of the two solutions. The fitted per-block-row slopes
show the linear-in-N cost of the direct method against the flat (until the
GPU is full) cost of PCG.

Run: python -m paper_2503_15269_amd.complexity [--quick] [--json]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

SINGLE_N = (8, 32, 128, 512, 2048, 8192, 32768)
BATCH_N = (16, 64, 256, 512)
WORKGROUP_CAPACITY = 8192  # unknowns per system of the batched kernels
QUICK_SINGLE_N = (16, 256)
QUICK_BATCH_N = (32,)


def _events_ms(torch, fn, reps=5, warmup=1):
    """Median event time of ``fn`` on the current stream."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return float(np.median(out))


def fit_slope(xs, ys):
    """Least-squares slope and intercept of ys against xs (per-unit cost)."""
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    if xs.size < 2:
        return float("nan"), float("nan")
    k, c = np.polyfit(xs, ys, 1)
    return float(k), float(c)


def crossover(rows, a, b):
    """Smallest N at which method ``b`` is faster than method ``a`` for good
    (faster there and at every larger N of the sweep); None if never."""
    best = None
    for r in sorted(rows, key=lambda r: -r["N"]):
        if r[b] < r[a]:
            best = r["N"]
        else:
            break
    return best


def _rel(x, y):
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def single_point(bt, torch, dev, N, n, nu, seed, tol, reps):
    import lqrgen
    d = lqrgen.lqr_instance(N, n, nu, seed, N)
    D = torch.tensor(d["D"], dtype=torch.float64, device=dev)
    O = torch.tensor(d["O"], dtype=torch.float64, device=dev)
    b = torch.tensor(d["b"].reshape(-1), dtype=torch.float64, device=dev)
    out = {"N": N, "n": n}
    hd = bt.Handle(D, O if N > 1 else None, None, bt.Params.polycoeff(2))
    xd, infd = hd.solve_direct(b)
    torch.cuda.synchronize()
    out["direct_ok"] = bool(bt.infos_to_numpy(infd)[0]["status"] == bt.OK)
    out["direct_ms"] = _events_ms(torch, lambda: hd.solve_direct(b, xd, infd),
                                  reps)
    xd_h = xd.cpu().numpy()
    for prec in ("f64", "f32_ir"):
        P = bt.Params.polycoeff(2, prec=prec)
        h = bt.Handle(D, O if N > 1 else None, None, P)
        x, info = h.solve_grid(b, tol)
        torch.cuda.synchronize()
        inf = bt.infos_to_numpy(info)[0]
        out[f"pcg_{prec}_ok"] = bool(inf["status"] == bt.OK)
        out[f"pcg_{prec}_iters"] = int(inf["iters"])
        out[f"pcg_{prec}_outer"] = int(inf["outer"])
        out[f"pcg_{prec}_rel_diff"] = _rel(x.cpu().numpy(), xd_h)
        out[f"pcg_{prec}_setup_ms"] = _events_ms(torch, h.refactor, reps)

        def step(h=h, x=x, info=info):
            h.refactor()
            h.solve_grid(b, tol, x=x, info=info)
        out[f"pcg_{prec}_grid_ms"] = _events_ms(torch, step, reps)
        # the single-workgroup path where the system fits one workgroup
        wg = None
        if N * n <= WORKGROUP_CAPACITY:
            xw, iw = h.solve(b, tol)
            torch.cuda.synchronize()
            if bt.infos_to_numpy(iw)[0]["status"] == bt.OK:
                def step_wg(h=h, x=xw, info=iw):
                    h.refactor()
                    h.solve(b, tol, x=x, info=info)
                wg = _events_ms(torch, step_wg, reps)
            del xw, iw
        out[f"pcg_{prec}_workgroup_ms"] = wg
        out[f"pcg_{prec}_ms"] = min(out[f"pcg_{prec}_grid_ms"],
                                    wg if wg is not None else float("inf"))
        del h, x, info
    return out


def batch_point(bt, torch, dev, B, N, n, nu, seed, tol, reps):
    import lqrgen
    data = lqrgen.lqr_batch(B, N, n, nu, seed)
    D = torch.tensor(data["D"], dtype=torch.float64, device=dev)
    O = torch.tensor(data["O"], dtype=torch.float64, device=dev)
    b = torch.tensor(data["b"].reshape(-1), dtype=torch.float64, device=dev)
    off = data["offsets"]
    out = {"N": N, "n": n, "B": B}
    hd = bt.Handle(D, O if N > 1 else None, off, bt.Params.polycoeff(2))
    xd, infd = hd.solve_direct(b)
    torch.cuda.synchronize()
    out["direct_ok"] = bool(np.all(bt.infos_to_numpy(infd)["status"] == bt.OK))
    out["direct_ms"] = _events_ms(torch, lambda: hd.solve_direct(b, xd, infd),
                                  reps)
    xd_h = xd.cpu().numpy()
    for prec in ("f64", "f32_ir"):
        P = bt.Params.polycoeff(2, prec=prec)
        h = bt.Handle(D, O if N > 1 else None, off, P)
        x, info = h.solve(b, tol)
        torch.cuda.synchronize()
        inf = bt.infos_to_numpy(info)
        out[f"pcg_{prec}_ok"] = bool(np.all(inf["status"] == bt.OK))
        out[f"pcg_{prec}_iters_mean"] = float(inf["iters"].mean())
        out[f"pcg_{prec}_rel_diff"] = _rel(x.cpu().numpy(), xd_h)

        def step(h=h, x=x, info=info):
            h.refactor()
            h.solve(b, tol, x=x, info=info)
        out[f"pcg_{prec}_ms"] = _events_ms(torch, step, reps)
        del h, x, info
    return out


def run(single_N=SINGLE_N, batch_N=BATCH_N, n=12, nu=4, B=512,
        seed=20250319, tol=1e-10, reps=5, verbose=False):
    import torch

    import paper_2503_15269_amd as bt
    bt.load_library()
    dev = torch.device("cuda:0")
    single, batch = [], []
    for N in single_N:
        single.append(single_point(bt, torch, dev, N, n, nu, seed, tol, reps))
        if verbose:
            print(json.dumps(single[-1]), flush=True)
    for N in batch_N:
        batch.append(batch_point(bt, torch, dev, B, N, n, nu, seed, tol,
                                 reps))
        if verbose:
            print(json.dumps(batch[-1]), flush=True)
    summary = {}
    for name, rows in (("single", single), ("batch", batch)):
        if not rows:
            continue
        Ns = [r["N"] for r in rows]
        s = {"direct_ms_per_block_row": fit_slope(Ns, [r["direct_ms"]
                                                       for r in rows])[0]}
        for prec in ("f64", "f32_ir"):
            s[f"pcg_{prec}_ms_per_block_row"] = fit_slope(
                Ns, [r[f"pcg_{prec}_ms"] for r in rows])[0]
            s[f"crossover_N_{prec}"] = crossover(rows, "direct_ms",
                                                 f"pcg_{prec}_ms")
        summary[name] = s
    return dict(n=n, nu=nu, B=B, tol=tol, seed=seed, single=single,
                batch=batch, summary=summary)


def markdown(res):
    out = [f"n = {res['n']}, nu = {res['nu']}, relative tolerance "
           f"{res['tol']:g}; times are whole calls (setup included), median "
           f"of several runs.", "",
           "One system:", "",
           "| N | direct ms | PCG f64 ms (iters) [grid / workgroup] | "
           "PCG f32+IR ms (iters, outer) [grid / workgroup] | "
           "direct / best PCG | max rel. diff |",
           "|---|---|---|---|---|---|"]

    def paths(r, prec):
        wg = r[f"pcg_{prec}_workgroup_ms"]
        return (f"[{r[f'pcg_{prec}_grid_ms']:.3f} / "
                f"{'-' if wg is None else format(wg, '.3f')}]")
    for r in res["single"]:
        best = min(r["pcg_f64_ms"], r["pcg_f32_ir_ms"])
        out.append(
            f"| {r['N']} | {r['direct_ms']:.3f} | {r['pcg_f64_ms']:.3f} "
            f"({r['pcg_f64_iters']}) {paths(r, 'f64')} | "
            f"{r['pcg_f32_ir_ms']:.3f} ({r['pcg_f32_ir_iters']}, "
            f"{r['pcg_f32_ir_outer']}) {paths(r, 'f32_ir')} | "
            f"{r['direct_ms'] / best:.2f} | "
            f"{max(r['pcg_f64_rel_diff'], r['pcg_f32_ir_rel_diff']):.1e} |")
    if res["batch"]:
        out += ["", f"Batch of {res['B']} systems:", "",
                "| N | direct ms | PCG f64 ms (mean iters) | PCG f32+IR ms "
                "(mean inner iters) | direct / best PCG | max rel. diff |",
                "|---|---|---|---|---|---|"]
        for r in res["batch"]:
            best = min(r["pcg_f64_ms"], r["pcg_f32_ir_ms"])
            out.append(
                f"| {r['N']} | {r['direct_ms']:.3f} | {r['pcg_f64_ms']:.3f} "
                f"({r['pcg_f64_iters_mean']:.1f}) | {r['pcg_f32_ir_ms']:.3f} "
                f"({r['pcg_f32_ir_iters_mean']:.1f}) | "
                f"{r['direct_ms'] / best:.2f} | "
                f"{max(r['pcg_f64_rel_diff'], r['pcg_f32_ir_rel_diff']):.1e} |")
    out += ["", "```", json.dumps(res["summary"], indent=1), "```"]
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--json", action="store_true")
    ap.add_argument("--batch", type=int, default=512)
    args = ap.parse_args()
    kw = dict(B=args.batch, verbose=args.json)
    if args.quick:
        kw.update(single_N=QUICK_SINGLE_N, batch_N=QUICK_BATCH_N, reps=3)
    print(markdown(run(**kw)), flush=True)


if __name__ == "__main__":
    main()
