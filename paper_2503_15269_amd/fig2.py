"""The paper's numerical experiment (Section V, Fig. 2) rerun on the GPU.

For each splitting family -- "Block Jacobi" (a, b) = (0, 1), "Equal"
(1/3, 1/3), "Stairs only" (1/2, 0), "Optimal" (1, -1) and "PolyCoeff"
(optimal weights with alpha_{m-1} = 7, Section V footnote) -- and each
polynomial order m = 1..4, random LQR Schur complements (N = 30 block rows,
n = 20) are solved by PCG for many right-hand sides. Reported per setting:
the mean PCG iteration count n_itr, the block-gemv count n_itr * g_a(m)
(Section IV-B), and, on a subset of the matrices, the smallest and largest
eigenvalue of M^{-1} A, the number of distinct eigenvalues and the condition
number relative to "Block Jacobi", m = 1.

Everything runs through the library: the solves are one batched launch per
setting (every matrix replicated once per right-hand side), and M^{-1} for
the spectra is formed column by column with bt_precondition. Eigenvalues of
the (small, dense) preconditioned matrices are computed with numpy.

The paper stops at an absolute residual of 1e-6; the library's test is
relative, so the tolerance is 1e-6 / sqrt(N n), the expected norm of a
standard normal right-hand side (their norms spread by a few per cent).

Run: python -m paper_2503_15269_amd.fig2 [--matrices 100] [--rhs 100]
     python -m paper_2503_15269_amd.fig2 --alpha-search 2   (alpha grid)
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

FAMILIES = (("Block Jacobi", 0.0, 1.0, False),
            ("Equal", 1.0 / 3.0, 1.0 / 3.0, False),
            ("Stairs only", 0.5, 0.0, False),
            ("Optimal", 1.0, -1.0, False),
            ("PolyCoeff", 1.0, -1.0, True))


def gemv_per_iteration(a: float, m: int) -> int:
    """g_a(m) of Section IV-B."""
    if a == 0.0:
        return 2 * m + 2
    if a == 1.0:
        return 3 * m + 3
    return 5 * m + 1


def params_for(bt, a, b, m, poly):
    alpha = bt.polycoeff(m) if poly else [1.0] * m
    return bt.Params(a=a, b=b, m=m, alpha=alpha, prec="f64")


def distinct_count(lam, rel=1e-6):
    """Number of clusters of the sorted eigenvalues (gap > rel * max)."""
    lam = np.sort(np.asarray(lam))
    if lam.size == 0:
        return 0
    gaps = np.diff(lam) > rel * max(abs(lam[-1]), 1e-300)
    return int(1 + np.count_nonzero(gaps))


def dense_A(D, O):
    N, n = D.shape[0], D.shape[1]
    A = np.zeros((N * n, N * n))
    for k in range(N):
        A[k * n:(k + 1) * n, k * n:(k + 1) * n] = D[k]
        if k + 1 < N:
            A[k * n:(k + 1) * n, (k + 1) * n:(k + 2) * n] = O[k]
            A[(k + 1) * n:(k + 2) * n, k * n:(k + 1) * n] = O[k].T
    return A


def run(matrices=100, rhs=100, N=30, n=20, nu=7, ms=(1, 2, 3, 4),
        eig_matrices=5, seed=20250502, verbose=False):
    import torch

    import lqrgen
    import paper_2503_15269_amd as bt
    from . import Handle, infos_to_numpy, OK

    dev = torch.device("cuda:0")
    insts = [lqrgen.lqr_instance(N, n, nu, seed, i, nrhs=rhs)
             for i in range(matrices)]
    B = matrices * rhs
    offs = np.arange(B + 1, dtype=np.int64) * N
    # system (i, j) = matrix i with right-hand side j, rows concatenated
    D_t = torch.tensor(np.stack([d["D"] for d in insts]), dtype=torch.float64,
                       device=dev).repeat_interleave(rhs, dim=0)
    O_t = torch.tensor(np.stack([d["O"] for d in insts]), dtype=torch.float64,
                       device=dev).repeat_interleave(rhs, dim=0)
    D_t = D_t.reshape(-1, n, n).contiguous()
    O_t = O_t.reshape(-1, n, n).contiguous()
    bb = np.stack([np.transpose(d["b"], (2, 0, 1)) for d in insts])
    b_t = torch.tensor(bb.reshape(-1), dtype=torch.float64, device=dev)
    tol = 1e-6 / np.sqrt(N * n)

    # one preconditioner application per unit vector gives M^{-1} column-wise
    eye = torch.eye(N * n, dtype=torch.float64, device=dev)
    A_dense = [dense_A(insts[i]["D"], insts[i]["O"]) for i in range(eig_matrices)]
    E_D = [torch.tensor(insts[i]["D"], dtype=torch.float64, device=dev)
           .repeat(N * n, 1, 1).contiguous() for i in range(eig_matrices)]
    E_O = [torch.tensor(insts[i]["O"], dtype=torch.float64, device=dev)
           .repeat(N * n, 1, 1).contiguous() for i in range(eig_matrices)]
    e_offs = np.arange(N * n + 1, dtype=np.int64) * N

    rows = []
    for name, a, b, poly in FAMILIES:
        for m in ms:
            if poly and m == 1:
                continue  # no alpha for m = 1: the same as "Optimal"
            P = params_for(bt, a, b, m, poly)
            t0 = time.perf_counter()
            h = Handle(D_t, O_t, offs, P)
            x, info = h.solve(b_t, tol)
            torch.cuda.synchronize()
            inf = infos_to_numpy(info)
            ok = bool(np.all(inf["status"] == OK))
            its = inf["iters"].astype(np.float64)
            del h, x
            lmin, lmax, dist, cond = [], [], [], []
            for i in range(eig_matrices):
                he = Handle(E_D[i], E_O[i], e_offs, P)
                Minv = he.precondition(eye.reshape(-1).contiguous())
                Minv = Minv.reshape(N * n, N * n).cpu().numpy().T  # columns
                lam = np.linalg.eigvals(Minv @ A_dense[i]).real
                lmin.append(lam.min())
                lmax.append(lam.max())
                dist.append(distinct_count(lam))
                cond.append(lam.max() / lam.min())
                del he
            rows.append(dict(family=name, a=a, b=b, m=m, converged=ok,
                             iters_mean=float(its.mean()),
                             iters_max=int(its.max()),
                             gemv_mean=float(its.mean()) * gemv_per_iteration(a, m),
                             lam_min=float(np.mean(lmin)),
                             lam_max=float(np.mean(lmax)),
                             distinct=float(np.mean(dist)),
                             cond=float(np.mean(cond)),
                             seconds=time.perf_counter() - t0))
            if verbose:
                print(json.dumps(rows[-1]), flush=True)
    ref = [r for r in rows if r["family"] == "Block Jacobi" and r["m"] == 1]
    c0 = ref[0]["cond"] if ref else 1.0
    for r in rows:
        r["cond_rel"] = r["cond"] / c0
    return dict(N=N, n=n, nu=nu, matrices=matrices, rhs=rhs,
                eig_matrices=eig_matrices, tol_rel=tol, rows=rows)


def alpha_search(alphas=(1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 15), m=2,
                 matrices=20, rhs=20, N=30, n=20, nu=7, seed=20250502):
    """Grid search of the last polynomial coefficient alpha_{m-1} at the
    optimal weights (the search behind the Section V footnote): mean PCG
    iterations and gemvs on the same random systems for each value (the
    other coefficients 1). Returns [(alpha, iters_mean, gemv_mean)]."""
    import torch

    import lqrgen
    import paper_2503_15269_amd as bt
    from . import Handle, infos_to_numpy, OK

    dev = torch.device("cuda:0")
    insts = [lqrgen.lqr_instance(N, n, nu, seed, i, nrhs=rhs)
             for i in range(matrices)]
    offs = np.arange(matrices * rhs + 1, dtype=np.int64) * N
    D_t = torch.tensor(np.stack([d["D"] for d in insts]), dtype=torch.float64,
                       device=dev).repeat_interleave(rhs, dim=0)
    O_t = torch.tensor(np.stack([d["O"] for d in insts]), dtype=torch.float64,
                       device=dev).repeat_interleave(rhs, dim=0)
    D_t = D_t.reshape(-1, n, n).contiguous()
    O_t = O_t.reshape(-1, n, n).contiguous()
    bb = np.stack([np.transpose(d["b"], (2, 0, 1)) for d in insts])
    b_t = torch.tensor(bb.reshape(-1), dtype=torch.float64, device=dev)
    tol = 1e-6 / np.sqrt(N * n)
    out = []
    for al in alphas:
        alpha = [1.0] * m
        if m > 1:
            alpha[m - 1] = float(al)
        P = bt.Params(a=1.0, b=-1.0, m=m, alpha=alpha, prec="f64")
        h = Handle(D_t, O_t, offs, P)
        x, info = h.solve(b_t, tol)
        torch.cuda.synchronize()
        inf = infos_to_numpy(info)
        its = inf["iters"].astype(np.float64)
        ok = bool(np.all(inf["status"] == OK))
        out.append((float(al), float(its.mean()) if ok else float("nan"),
                    float(its.mean()) * gemv_per_iteration(1.0, m)
                    if ok else float("nan")))
        del h, x
    return out


def markdown(res):
    out = [f"N = {res['N']}, n = {res['n']}, nu = {res['nu']}; "
           f"{res['matrices']} matrices x {res['rhs']} right-hand sides per "
           f"setting (spectra: first {res['eig_matrices']} matrices); "
           f"relative tolerance {res['tol_rel']:.3g}.", "",
           "| family | m | PCG iterations (mean / max) | block gemvs n_itr g_a(m) | "
           "min eig | max eig | distinct eigenvalues | cond / cond(BJ, m=1) |",
           "|---|---|---|---|---|---|---|---|"]
    for r in res["rows"]:
        out.append(f"| {r['family']} | {r['m']} | {r['iters_mean']:.2f} / "
                   f"{r['iters_max']} | {r['gemv_mean']:.1f} | "
                   f"{r['lam_min']:.3g} | {r['lam_max']:.4g} | "
                   f"{r['distinct']:.1f} | {r['cond_rel']:.3g} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--matrices", type=int, default=100)
    ap.add_argument("--rhs", type=int, default=100)
    ap.add_argument("--eig-matrices", type=int, default=5)
    ap.add_argument("--json", action="store_true")
    ap.add_argument("--alpha-search", type=int, default=0, metavar="M",
                    help="instead: grid search of alpha_{M-1} at order M")
    args = ap.parse_args()
    if args.alpha_search:
        m = args.alpha_search
        rows = alpha_search(m=m)
        print(f"| alpha_{m - 1} | PCG iterations (mean) | block gemvs |")
        print("|---|---|---|")
        for al, it, gv in rows:
            print(f"| {al:g} | {it:.2f} | {gv:.1f} |")
        return
    res = run(matrices=args.matrices, rhs=args.rhs,
              eig_matrices=args.eig_matrices, verbose=args.json)
    print(markdown(res))


if __name__ == "__main__":
    main()
