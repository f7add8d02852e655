"""Stagnating float32 refinement: a system whose conditioning is beyond the
float32 operator (kappa ~ 1e10; the float32 refinement still converges at
kappa 1e8-1e9 on these systems) stops with ESTAGNATED on every refinement
path instead of running out its refinement steps; with fallback_f64 the
batched solve finishes it in float64 on the device (same call, same
stream), while the other systems of the batch keep their float32 result
bit for bit."""
import numpy as np
import pytest

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt
from dense import dense_A
from gpu_util import assert_close, to_dev, true_relres

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bt.load_library()


def ill_conditioned(N, n, seed, kappa):
    """An LQR Schur complement with its spectrum shifted so that
    lambda_min = lambda_max / kappa (every diagonal block moved by the same
    multiple of I: still SPD and block tridiagonal)."""
    d = lqrgen.lqr_instance(N, n, max(1, n // 3), seed, 0, s=0.1)
    D, O = d["D"].copy(), d["O"]
    ev = np.linalg.eigvalsh(dense_A(D, O))
    shift = ev[0] - ev[-1] / kappa
    D -= shift * np.eye(n)
    return D, O, d["b"]


KAPPA = 1e10


def batch(n, ill_at, N=24, kappa=KAPPA):
    """Six systems of N block rows; the ones in ``ill_at`` ill-conditioned."""
    Ds, Os, bs = [], [], []
    for i in range(6):
        if i in ill_at:
            D, O, b = ill_conditioned(N, n, 500 + i, kappa)
        else:
            d = lqrgen.lqr_instance(N, n, max(1, n // 3), 500 + i, 0, s=0.1)
            D, O, b = d["D"], d["O"], d["b"]
        Ds.append(D)
        Os.append(O)
        bs.append(b)
    off = np.arange(7, dtype=np.int64) * N
    return np.concatenate(Ds), np.concatenate(Os), np.concatenate(bs), off


def solve(D, O, b, off, fallback, tol):
    import torch
    P = bt.Params.polycoeff(2, prec="f32_ir", inner_tol=1e-4,
                            fallback_f64=fallback)
    h = bt.Handle(to_dev(D, torch.float64), to_dev(O, torch.float64), off, P)
    x, info = h.solve(to_dev(b.reshape(-1), torch.float64), tol)
    torch.cuda.synchronize()
    return x.cpu().numpy().reshape(D.shape[0], -1), bt.infos_to_numpy(info), h


@pytest.mark.parametrize("n", [12, 8])   # register-resident / generic kernel
def test_stagnation_reported_without_fallback(n):
    D, O, b, off = batch(n, ill_at=(1, 4))
    x, info, h = solve(D, O, b, off, False, 1e-5)
    if n == 12:
        assert h.kernel_config() >= bt.load_library().bt_kernel_config_count() - 3
    for i in range(6):
        if i in (1, 4):
            assert info[i]["status"] == bt.ESTAGNATED, info[i]
            assert 1 <= info[i]["outer"] <= 4, info[i]   # no run to max_outer
        else:
            assert info[i]["status"] == bt.OK, info[i]


@pytest.mark.parametrize("n", [12, 8])
def test_fallback_finishes_in_float64(n):
    """With fallback_f64 the stagnated systems end BT_OK in float64, their
    counts adding the float32 steps; the others are left exactly as the
    float32 solve returned them. At kappa = 1e10 the float64 iteration's
    recursive residual (its stopping test) and the true residual drift apart
    by about u kappa ~ 1e-6, so the true residual is held to 2 tol."""
    D, O, b, off = batch(n, ill_at=(1, 4))
    tol = 1e-5
    x0, info0, _ = solve(D, O, b, off, False, tol)
    x, info, _ = solve(D, O, b, off, True, tol)
    for i in range(6):
        rows = slice(int(off[i]), int(off[i + 1]))
        oblk = slice(int(off[i]) - i, int(off[i + 1]) - i - 1)
        assert info[i]["status"] == bt.OK, info[i]
        if i in (1, 4):
            assert info0[i]["status"] == bt.ESTAGNATED
            assert true_relres(D[rows], O[oblk], b[rows], x[rows]) <= 2 * tol
            assert info[i]["outer"] == info0[i]["outer"] + 1
            assert info[i]["iters"] > info0[i]["iters"]
            assert info[i]["gemv_paper"] > info0[i]["gemv_paper"]
        else:
            assert np.array_equal(x[rows], x0[rows])
            assert info[i]["iters"] == info0[i]["iters"]
            assert true_relres(D[rows], O[oblk], b[rows], x[rows]) <= tol
            xd = orc.btchol_solve(D[rows], O[oblk], b[rows])
            assert_close(x[rows], xd, 1e-5, i)


def test_fallback_idle_on_well_conditioned_batches():
    """Nothing stagnates: the fallback passes only read the statuses, and the
    results equal those of the same solve without them."""
    D, O, b, off = batch(12, ill_at=())
    x0, info0, _ = solve(D, O, b, off, False, 1e-10)
    x, info, _ = solve(D, O, b, off, True, 1e-10)
    assert np.all(info["status"] == bt.OK)
    assert np.array_equal(x, x0)
    assert np.array_equal(info["iters"], info0["iters"])


def test_stagnation_on_the_grid_path():
    import torch
    D, O, b = ill_conditioned(48, 12, 77, KAPPA)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    h = bt.Handle(to_dev(D, torch.float64), to_dev(O, torch.float64), None, P)
    x, info = h.solve_grid(to_dev(b.reshape(-1), torch.float64), 1e-5)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)
    assert inf[0]["status"] == bt.ESTAGNATED and 1 <= inf[0]["outer"] <= 4, inf


def test_stagnation_on_the_multi_rhs_path():
    import torch
    D, O, _ = ill_conditioned(16, 16, 78, KAPPA)
    rng = np.random.default_rng(3)
    B = rng.standard_normal((16, 16, 16))
    h = bt.Handle(to_dev(D, torch.float64), to_dev(O, torch.float64), None,
                  bt.Params.polycoeff(2, prec="bf16x2_ir"))
    X, info = h.solve_mrhs(to_dev(B, torch.float64), 1e-5)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)
    assert np.all(inf["status"] == bt.ESTAGNATED), inf["status"]
    assert np.all(inf["outer"] <= 4)
