"""Many right-hand sides on the matrix cores (BF16 hi/lo split blocks, float32
accumulation, float64 refinement) against the oracle's direct solve, per
right-hand side."""
import numpy as np
import pytest

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt
from gpu_util import rowmax_rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bt.load_library()


def run_mrhs(N, n, nu, nrhs, seed, s=0.05, tol=1e-10, m=2, record="f32"):
    import torch
    d = lqrgen.lqr_instance(N, n, nu, seed, 0, s=s, nrhs=nrhs)
    D, O, B = d["D"], d["O"], d["b"]
    if record == "f32":
        D = D.astype(np.float32).astype(np.float64)
        O = O.astype(np.float32).astype(np.float64)
    dt = torch.float32 if record == "f32" else torch.float64
    h = bt.Handle(to_dev(D, dt), to_dev(O, dt), None,
                  bt.Params.polycoeff(m, prec="bf16x2_ir", inner_tol=1e-4))
    X, info = h.solve_mrhs(to_dev(B, torch.float64), tol)
    torch.cuda.synchronize()
    return D, O, B, X.cpu().numpy(), bt.infos_to_numpy(info)


def check(D, O, B, X, info, tol=1e-10, err_bound=2e-5, cols=None):
    assert np.all(info["status"] == bt.OK), np.unique(info["status"])
    assert np.all(info["relres_true"] <= tol)
    Xd = orc.btchol_solve(D, O, B)
    for c in (range(B.shape[2]) if cols is None else cols):
        r = B[:, :, c] - orc.spmv(D, O, X[:, :, c])
        assert np.linalg.norm(r) <= 1.01 * tol * np.linalg.norm(B[:, :, c]), c
        err = np.linalg.norm(X[:, :, c] - Xd[:, :, c]) / np.linalg.norm(Xd[:, :, c])
        assert err <= err_bound, (c, err)
        row = rowmax_rel(X[:, :, c], Xd[:, :, c])
        assert row <= err_bound, (c, "row max", row)


@pytest.mark.parametrize("m", [1, 2])
def test_mrhs_n48_small(m):
    D, O, B, X, info = run_mrhs(40, 48, 16, 64, seed=5, m=m)
    check(D, O, B, X, info)


def test_mrhs_n64():
    """n = 64: every product takes two K steps of 32 (the 32-deep bfloat16
    form over pairs of panel tiles)."""
    D, O, B, X, info = run_mrhs(20, 64, 21, 64, seed=9)
    check(D, O, B, X, info)


def test_mrhs_n16_two_column_blocks():
    D, O, B, X, info = run_mrhs(33, 16, 5, 128, seed=6, s=0.1)
    check(D, O, B, X, info)


def test_mrhs_f64_record_and_zero_column():
    import torch
    d = lqrgen.lqr_instance(20, 32, 8, 8, 0, s=0.1, nrhs=64)
    B = d["b"].copy()
    B[:, :, 5] = 0.0
    h = bt.Handle(to_dev(d["D"], torch.float64), to_dev(d["O"], torch.float64),
                  None, bt.Params.polycoeff(2, prec="bf16x2_ir"))
    X, info = h.solve_mrhs(to_dev(B, torch.float64), 1e-10)
    inf = bt.infos_to_numpy(info)
    X = X.cpu().numpy()
    assert inf[5]["status"] == bt.OK and inf[5]["iters"] == 0
    assert not np.any(X[:, :, 5])
    check(d["D"], d["O"], B, X, inf, cols=[0, 1, 17, 63])


def test_mrhs_argument_checks():
    import torch
    d = lqrgen.lqr_instance(8, 16, 4, 1, 0, nrhs=64)
    Dt, Ot = to_dev(d["D"], torch.float64), to_dev(d["O"], torch.float64)
    B = to_dev(d["b"], torch.float64)
    h = bt.Handle(Dt, Ot, None, bt.Params.polycoeff(2, prec="f32_ir"))
    with pytest.raises(bt.BtError):
        h.solve_mrhs(B)                      # handle not set up for bf16x2
    h2 = bt.Handle(Dt, Ot, None, bt.Params.polycoeff(2, prec="bf16x2_ir"))
    with pytest.raises(bt.BtError):
        h2.solve_mrhs(B[:, :, :24].contiguous())   # nrhs not a multiple of 16
    h3 = bt.Handle(Dt, Ot, None, bt.Params(pc="none", m=1, prec="bf16x2_ir"))
    with pytest.raises(bt.BtError):
        h3.solve_mrhs(B)                     # no preconditioner: not here


@pytest.mark.parametrize("scale", [1e-14, 1e18])
def test_mrhs_scaled_columns(scale):
    """Columns far from unit scale: the float32 inner solves see each
    column's residual scaled to unit norm, so tiny and huge right-hand sides
    converge like unit ones."""
    import torch
    d = lqrgen.lqr_instance(40, 48, 16, 31, 0, s=0.05, nrhs=64)
    D = d["D"].astype(np.float32).astype(np.float64)
    O = d["O"].astype(np.float32).astype(np.float64)
    B = d["b"].copy()
    B[:, :, ::2] *= scale   # every other column scaled
    h = bt.Handle(to_dev(D, torch.float32), to_dev(O, torch.float32), None,
                  bt.Params.polycoeff(2, prec="bf16x2_ir", inner_tol=1e-4))
    X, info = h.solve_mrhs(to_dev(B, torch.float64), 1e-10)
    torch.cuda.synchronize()
    check(D, O, B, X.cpu().numpy(), bt.infos_to_numpy(info))


# Preconditioners of the whole family (the fused kernels cover a = 1, m <= 2;
# the rest goes through the Horner passes), nrhs multiples of 16 that leave
# a workgroup's last columns past the panel.
GENERAL = [(0.0, 1, None, 16, 16), (0.0, 3, [1.0, 0.5, 2.0], 48, 32),
           (0.5, 2, [1.0, 3.0], 80, 16), (0.5, 4, [1.0, 1.0, 1.0, 7.0], 48, 48),
           (1.0, 3, [1.0, 1.0, 7.0], 144, 32), (1.0, 4, [1.0, 2.0, 1.0, 7.0], 16, 16),
           (1.0, 2, [1.0, 7.0], 48, 48)]


def _params(a, m, alpha, **kw):
    return bt.Params(a=a, m=m, alpha=alpha, prec="bf16x2_ir", **kw)


@pytest.mark.parametrize("a,m,alpha,nrhs,n", GENERAL)
def test_mrhs_general_first_step(a, m, alpha, nrhs, n):
    """One inner iteration from x = 0 (maxit = 1) leaves X = alpha_0 z with
    z = M^{-1} b the oracle's preconditioner (any splitting, order and
    coefficients) and alpha_0 = b'z / z'Az: this pins the preconditioner the
    panel passes evaluate, column by column, to the precision of the
    bfloat16-pair products (~1e-5)."""
    import torch
    d = lqrgen.lqr_instance(24, n, max(1, n // 3), 70 + n, 0, s=0.1, nrhs=nrhs)
    D, O, B = d["D"], d["O"], d["b"]
    h = bt.Handle(to_dev(D, torch.float64), to_dev(O, torch.float64), None,
                  _params(a, m, alpha, max_outer=1))
    X, info = h.solve_mrhs(to_dev(B, torch.float64), 1e-10, maxit=1)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    inf = bt.infos_to_numpy(info)
    assert np.all(inf["iters"] == 1)
    for c in range(nrhs):
        b = B[:, :, c]
        kind = orc.PC_OPT if a == 1.0 else orc.PC_SPLIT
        z = orc.precond(D, O, b, kind=kind, a=a, b=1.0 - 2.0 * a, m=m,
                        alpha=alpha)
        x1 = (np.sum(b * z) / np.sum(z * orc.spmv(D, O, z))) * z
        err = np.linalg.norm(X[:, :, c] - x1) / np.linalg.norm(x1)
        assert err <= 1e-3, (c, err)


@pytest.mark.parametrize("a,m,alpha,nrhs,n", GENERAL)
def test_mrhs_general_converges(a, m, alpha, nrhs, n):
    """Full solves to 1e-10 with every preconditioner of the family: every
    column's true residual and its error against the oracle's direct solve,
    and the gemv counts (the paper's g_a(m) per inner iteration)."""
    import torch
    d = lqrgen.lqr_instance(30, n, max(1, n // 3), 90 + n, 0, s=0.1, nrhs=nrhs)
    D = d["D"].astype(np.float32).astype(np.float64)
    O = d["O"].astype(np.float32).astype(np.float64)
    B = d["b"]
    h = bt.Handle(to_dev(D, torch.float32), to_dev(O, torch.float32), None,
                  _params(a, m, alpha, inner_tol=1e-4))
    X, info = h.solve_mrhs(to_dev(B, torch.float64), 1e-10)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)
    check(D, O, B, X.cpu().numpy(), inf)
    g = orc.gemv_per_iteration(orc.PC_SPLIT if a != 1.0 else orc.PC_OPT,
                               a=a, m=m)
    assert np.all(inf["gemv_paper"] == g * inf["iters"])
