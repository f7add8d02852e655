"""The standard workloads at full size, at every setting bench.py may time:
every system converges to the float64 tolerance, sampled systems agree with
the oracle's direct solve (globally and per block row), gradients agree with
the oracle's gradient and with central finite differences of the oracle's
direct solve. bench.py picks the kernel configuration and the inner
tolerance by timing them on the box, so each candidate inner tolerance is
checked here."""
import functools

import numpy as np
import pytest

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt
from gpu_util import (F64_TRUE_RES, assert_close, rel, to_dev, true_relres,
                      workload)
from paper_2503_15269_amd import autotune

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bt.load_library()


@functools.lru_cache(maxsize=None)
def _data(name):
    return workload(name)


@functools.lru_cache(maxsize=None)
def _ragged_direct(i):
    data = _data("batch_ragged_n12")
    r0, r1 = int(data["offsets"][i]), int(data["offsets"][i + 1])
    return orc.btchol_solve(data["D"][r0:r1], data["O"][r0 - i:r1 - i - 1],
                            data["b"][r0:r1])


def _fast_configs():
    first = bt.load_library().bt_kernel_config_count() - 3
    return [first, first + 1]   # 3 and 6 entries per lane (the tuned ones)


@pytest.mark.parametrize("itol", autotune.INNER_TOLS)
@pytest.mark.parametrize("variant", [0, 1])
def test_batch_ragged_n12_full(itol, variant):
    """2048 ragged systems, n = 12, float32 record, float32 inner PCG at each
    candidate inner tolerance and each register-resident variant the
    autotuner weighs."""
    import torch
    data = _data("batch_ragged_n12")
    D = to_dev(data["D"], torch.float32)
    O = to_dev(data["O"], torch.float32)
    b = to_dev(data["b"].reshape(-1), torch.float64)
    P = bt.Params.polycoeff(2, prec="f32_ir", inner_tol=itol)
    h = bt.Handle(D, O, data["offsets"], P)
    h.set_kernel_config(_fast_configs()[variant])
    x, info = h.solve(b, 1e-10)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)
    x = x.cpu().numpy().reshape(-1, 12)
    assert np.all(inf["status"] == bt.OK)
    assert np.all(inf["relres_true"] <= 1e-10)
    assert np.all(inf["gemv_paper"] == 9 * inf["iters"])
    rng = np.random.default_rng(0)
    for i in rng.choice(len(data["horizons"]), 24, replace=False):
        r0, r1 = int(data["offsets"][i]), int(data["offsets"][i + 1])
        Di, Oi, bi = data["D"][r0:r1], data["O"][r0 - i:r1 - i - 1], data["b"][r0:r1]
        assert true_relres(Di, Oi, bi, x[r0:r1]) <= F64_TRUE_RES
        assert_close(x[r0:r1], _ragged_direct(int(i)), 1e-7, int(i))


def _fd_ok(fd_h, fd_2h, g):
    """Acceptance of a central difference: within 1e-5 relative of the
    gradient, or within four times the difference between the steps h and
    2h (the truncation and rounding error of the difference itself)."""
    return abs(fd_h - g) <= max(1e-5 * abs(g), 4 * abs(fd_h - fd_2h))


@pytest.mark.parametrize("itol", autotune.INNER_TOLS)
def test_batch_grad_n24_full(itol):
    """256 systems, N = 128, n = 24, float32 record with refinement at each
    candidate inner tolerance of the timed forward + adjoint:
    L = sum ||x_k - t_k||^2, gradients for b, D, O against the oracle's
    gradient on sampled systems and central differences (h = 1e-6) of the
    oracle's direct solve on 20 random entries."""
    import torch
    data = _data("batch_grad_n24")
    D, O, b, t = data["D"], data["O"], data["b"], data["t"]
    Dt = torch.tensor(D, dtype=torch.float32, device="cuda", requires_grad=True)
    Ot = torch.tensor(O, dtype=torch.float32, device="cuda", requires_grad=True)
    btn = torch.tensor(b, dtype=torch.float64, device="cuda", requires_grad=True)
    tt = torch.tensor(t, dtype=torch.float64, device="cuda")
    P = bt.Params.polycoeff(2, prec="f32_ir", inner_tol=itol)
    x = bt.bt_solve(Dt, Ot, btn, data["offsets"], P, tol=1e-10)
    loss = ((x - tt) ** 2).sum()
    loss.backward()
    gD, gO, gb = Dt.grad.cpu().numpy(), Ot.grad.cpu().numpy(), btn.grad.cpu().numpy()
    xs = x.detach().cpu().numpy()
    rng = np.random.default_rng(lqrgen.workload_seed(3))
    for i in rng.choice(256, 4, replace=False):
        rows = slice(128 * i, 128 * (i + 1))
        oblk = slice(127 * i, 127 * (i + 1))
        assert true_relres(D[rows], O[oblk], b[rows], xs[rows]) <= F64_TRUE_RES
        xo = orc.btchol_solve(D[rows], O[oblk], b[rows])
        lam, dD, dO = orc.adjoint(D[rows], O[oblk], xo, 2 * (xo - t[rows]))
        assert_close(gb[rows], lam, 1e-5, ("dL/db", i))
        assert_close(gD[rows].reshape(-1, 24 * 24), dD.reshape(-1, 24 * 24),
                     1e-5, ("dL/dD", i))
        assert_close(gO[oblk].reshape(-1, 24 * 24), dO.reshape(-1, 24 * 24),
                     1e-5, ("dL/dO", i))
    # central differences of the oracle's direct solve on 20 random entries
    i = int(rng.integers(256))
    rows = slice(128 * i, 128 * (i + 1))
    oblk = slice(127 * i, 127 * (i + 1))
    Di, Oi, bi, ti = D[rows].copy(), O[oblk].copy(), b[rows].copy(), t[rows]

    def loss_of(D_, O_, b_):
        x_ = orc.btchol_solve(D_, O_, b_)
        return float(np.sum((x_ - ti) ** 2))

    def central(which, k, a_, c_, h):
        if which == 0:
            bp, bm = bi.copy(), bi.copy()
            bp[k, a_] += h
            bm[k, a_] -= h
            return (loss_of(Di, Oi, bp) - loss_of(Di, Oi, bm)) / (2 * h)
        if which == 1:   # D_k stays symmetric: move the pair together
            Dp, Dm = Di.copy(), Di.copy()
            for M, s in ((Dp, h), (Dm, -h)):
                M[k, a_, c_] += s
                if a_ != c_:
                    M[k, c_, a_] += s
            return (loss_of(Dp, Oi, bi) - loss_of(Dm, Oi, bi)) / (2 * h)
        Op, Om = Oi.copy(), Oi.copy()
        Op[k, a_, c_] += h
        Om[k, a_, c_] -= h
        return (loss_of(Di, Op, bi) - loss_of(Di, Om, bi)) / (2 * h)

    h = 1e-6
    for _ in range(20):
        which = int(rng.integers(3))
        k = int(rng.integers(127 if which == 2 else 128))
        a_, c_ = int(rng.integers(24)), int(rng.integers(24))
        if which == 0:
            g = gb[rows][k, a_]
        elif which == 1:
            g = gD[rows][k, a_, c_] + (gD[rows][k, c_, a_] if a_ != c_ else 0.0)
        else:
            g = gO[oblk][k, a_, c_]
        fd_h, fd_2h = central(which, k, a_, c_, h), central(which, k, a_, c_, 2 * h)
        assert _fd_ok(fd_h, fd_2h, g), (which, k, a_, c_, fd_h, fd_2h, g)


@functools.lru_cache(maxsize=None)
def _mrhs_direct():
    d = _data("multirhs_n48")
    D32 = d["D"].astype(np.float32).astype(np.float64)
    O32 = d["O"].astype(np.float32).astype(np.float64)
    return D32, O32, orc.btchol_solve(D32, O32, d["b"])


@pytest.mark.parametrize("itol", autotune.MRHS_INNER_TOLS)
def test_multirhs_n48_full(itol):
    """N = 4096, n = 48, 64 right-hand sides, BF16 split blocks on the matrix
    cores, float64 refinement, at each candidate inner tolerance: every
    column's true residual and its error against the direct solve."""
    import torch
    d = _data("multirhs_n48")
    D32, O32, Xd = _mrhs_direct()
    B = d["b"]
    h = bt.Handle(to_dev(D32, torch.float32), to_dev(O32, torch.float32), None,
                  bt.Params.polycoeff(2, prec="bf16x2_ir", inner_tol=itol))
    X, info = h.solve_mrhs(to_dev(B, torch.float64), 1e-10)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)
    X = X.cpu().numpy()
    assert np.all(inf["status"] == bt.OK), inf
    assert np.all(inf["relres_true"] <= 1e-10)
    for c in range(64):
        assert true_relres(D32, O32, B[:, :, c], X[:, :, c]) <= F64_TRUE_RES, c
        assert_close(X[:, :, c], Xd[:, :, c], 1e-7, c)
