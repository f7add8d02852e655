"""The standard workloads at full size, in the configuration bench.py times:
every system converges to the float64 tolerance, sampled systems agree with
the oracle's direct solve, gradients agree with the oracle's gradient and with
central finite differences of the oracle's direct solve."""
import numpy as np
import pytest

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt
from gpu_util import rel, to_dev, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bt.load_library()


def test_batch_ragged_n12_full():
    import torch
    from paper_2503_15269_amd import autotune
    data = workload("batch_ragged_n12")
    D = to_dev(data["D"], torch.float32)
    O = to_dev(data["O"], torch.float32)
    b = to_dev(data["b"].reshape(-1), torch.float64)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    tuned = autotune.tune(D, O, data["offsets"], b, P, 1e-10, reps=1,
                          use_cache=False)
    h = bt.Handle(D, O, data["offsets"], tuned["params"])
    h.set_kernel_config(tuned["kernel_config"])
    x, info = h.solve(b, 1e-10)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)
    x = x.cpu().numpy().reshape(-1, 12)
    assert np.all(inf["status"] == bt.OK)
    assert np.all(inf["relres_true"] <= 1e-10)
    rng = np.random.default_rng(0)
    for i in rng.choice(len(data["horizons"]), 24, replace=False):
        r0, r1 = int(data["offsets"][i]), int(data["offsets"][i + 1])
        Di, Oi, bi = data["D"][r0:r1], data["O"][r0 - i:r1 - i - 1], data["b"][r0:r1]
        r = bi - orc.spmv(Di, Oi, x[r0:r1])
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(bi)
        assert rel(x[r0:r1], orc.btchol_solve(Di, Oi, bi)) <= 1e-7


def test_batch_grad_n24_full():
    """256 systems, N = 128, n = 24, float32 record with refinement:
    L = sum ||x_k - t_k||^2, gradients for b, D, O."""
    import torch
    data = workload("batch_grad_n24")
    D, O, b, t = data["D"], data["O"], data["b"], data["t"]
    Dt = torch.tensor(D, dtype=torch.float32, device="cuda", requires_grad=True)
    Ot = torch.tensor(O, dtype=torch.float32, device="cuda", requires_grad=True)
    btn = torch.tensor(b, dtype=torch.float64, device="cuda", requires_grad=True)
    tt = torch.tensor(t, dtype=torch.float64, device="cuda")
    P = bt.Params.polycoeff(2, prec="f32_ir", inner_tol=1e-5)
    x = bt.bt_solve(Dt, Ot, btn, data["offsets"], P, tol=1e-10)
    loss = ((x - tt) ** 2).sum()
    loss.backward()
    gD, gO, gb = Dt.grad.cpu().numpy(), Ot.grad.cpu().numpy(), btn.grad.cpu().numpy()
    rng = np.random.default_rng(lqrgen.workload_seed(3))
    for i in rng.choice(256, 4, replace=False):
        rows = slice(128 * i, 128 * (i + 1))
        oblk = slice(127 * i, 127 * (i + 1))
        xo = orc.btchol_solve(D[rows], O[oblk], b[rows])
        lam, dD, dO = orc.adjoint(D[rows], O[oblk], xo, 2 * (xo - t[rows]))
        assert rel(gb[rows], lam) <= 1e-5
        assert rel(gD[rows], dD) <= 1e-5
        assert rel(gO[oblk], dO) <= 1e-5
    # central differences of the oracle's direct solve on 20 random entries
    i = int(rng.integers(256))
    rows = slice(128 * i, 128 * (i + 1))
    oblk = slice(127 * i, 127 * (i + 1))
    Di, Oi, bi, ti = D[rows].copy(), O[oblk].copy(), b[rows].copy(), t[rows]

    def loss_of(D_, O_, b_):
        x_ = orc.btchol_solve(D_, O_, b_)
        return float(np.sum((x_ - ti) ** 2))

    h = 1e-6
    for _ in range(20):
        which = rng.integers(3)
        if which == 0:
            k, a_ = rng.integers(128), rng.integers(24)
            bp, bm = bi.copy(), bi.copy()
            bp[k, a_] += h
            bm[k, a_] -= h
            fd = (loss_of(Di, Oi, bp) - loss_of(Di, Oi, bm)) / (2 * h)
            g = gb[rows][k, a_]
        elif which == 1:
            k, a_, c_ = rng.integers(128), rng.integers(24), rng.integers(24)
            Dp, Dm = Di.copy(), Di.copy()
            for M, s in ((Dp, h), (Dm, -h)):
                M[k, a_, c_] += s
                if a_ != c_:
                    M[k, c_, a_] += s
            fd = (loss_of(Dp, Oi, bi) - loss_of(Dm, Oi, bi)) / (2 * h)
            g = gD[rows][k, a_, c_] + (gD[rows][k, c_, a_] if a_ != c_ else 0.0)
        else:
            k, a_, c_ = rng.integers(127), rng.integers(24), rng.integers(24)
            Op, Om = Oi.copy(), Oi.copy()
            Op[k, a_, c_] += h
            Om[k, a_, c_] -= h
            fd = (loss_of(Di, Op, bi) - loss_of(Di, Om, bi)) / (2 * h)
            g = gO[oblk][k, a_, c_]
        assert abs(fd - g) <= max(1e-4 * abs(g), 1e-4), (which, fd, g)


def test_multirhs_n48_full():
    """N = 4096, n = 48, 64 right-hand sides, BF16 split blocks on the matrix
    cores, float64 refinement: per right-hand side residual and error."""
    import torch
    d = workload("multirhs_n48")
    D, O, B = d["D"], d["O"], d["b"]
    h = bt.Handle(to_dev(D, torch.float32), to_dev(O, torch.float32), None,
                  bt.Params.polycoeff(2, prec="bf16x2_ir", inner_tol=1e-4))
    X, info = h.solve_mrhs(to_dev(B, torch.float64), 1e-10)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)
    X = X.cpu().numpy()
    assert np.all(inf["status"] == bt.OK), inf
    assert np.all(inf["relres_true"] <= 1e-10)
    Xd = orc.btchol_solve(D, O, B)
    for c in range(64):
        r = B[:, :, c] - orc.spmv(D, O, X[:, :, c])
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(B[:, :, c])
        assert rel(X[:, :, c], Xd[:, :, c]) <= 1e-7
