"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

FP64: iteration counts equal the oracle's (off by one only when the oracle's
own stopping test sat within 1e-6 of its threshold) and solutions agree with
the oracle's PCG iterate to 1e-10 relative. FP32 + FP64 refinement: the
float64 residual of the record reaches the tolerance and the error against
the oracle's direct solve stays within the conditioning bound.
"""
import numpy as np
import pytest

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt
from gpu_util import (F64_TRUE_RES, assert_close, gpu_solve, iteration_match,
                      oracle_kind, rel, rowmax_rel, to_dev, true_relres,
                      workload)

pytestmark = pytest.mark.gpu

VARIANTS = {
    "polycoeff_m1": bt.Params.polycoeff(1),
    "polycoeff_m2": bt.Params.polycoeff(2),
    "polycoeff_m3": bt.Params.polycoeff(3),
    "polycoeff_m4": bt.Params.polycoeff(4),
    "opt_m2_alpha1": bt.Params(a=1.0, m=2),
    "jacobi_m1": bt.Params.block_jacobi(1),
    "jacobi_m2": bt.Params.block_jacobi(2),
    "stairs_m2": bt.Params(a=0.5, m=2),
    "equal_m3": bt.Params(a=1 / 3, m=3),
    "none": bt.Params(pc="none", m=1),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bt.load_library()


def _check_f64(D, O, b, params, tol=1e-10, xtol=1e-10):
    x, info, _ = gpu_solve(D, O, b, params=params, tol=tol)
    xr, ri = orc.pcg(D, O, b, tol=tol, maxit=10 * D.shape[0] * D.shape[1],
                     **oracle_kind(params))
    assert ri["status"] == orc.OK
    assert info[0]["status"] == bt.OK, info
    # plain CG (no preconditioner, hundreds of iterations) has lost
    # orthogonality and its count depends on rounding order: 1% slack there;
    # every preconditioner of the paper must match exactly
    slack = ri["iters"] // 100 if params.pc == "none" else 0
    assert iteration_match(int(info[0]["iters"]), ri, slack=slack), (info, ri)
    if info[0]["iters"] == ri["iters"]:
        assert_close(x, xr, xtol, "against the oracle's PCG iterate")
    elif slack:
        # both are converged iterates; they agree to the conditioning bound
        xd = orc.btchol_solve(D, O, b)
        assert_close(x, xd, 1e-6, "against the direct solve")
    assert info[0]["relres"] <= tol
    # the true residual of the returned x, from the oracle's product
    assert true_relres(D, O, b, x) <= 1.01 * tol
    assert info[0]["relres_true"] <= 1.01 * tol
    return x, info, ri


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_single_n6_f64_all_variants(name):
    d = workload("single_n6")
    _check_f64(d["D"], d["O"], d["b"], VARIANTS[name])


@pytest.mark.parametrize("name", ["polycoeff_m2", "polycoeff_m3", "jacobi_m1",
                                  "none"])
def test_single_n12_f64(name):
    d = workload("single_n12")
    _check_f64(d["D"], d["O"], d["b"], VARIANTS[name])


def test_single_n12_f32_refinement():
    d = workload("single_n12")
    P = bt.Params.polycoeff(2, prec="f32_ir")
    x, info, _ = gpu_solve(d["D"], d["O"], d["b"], params=P, tol=1e-10)
    assert info[0]["status"] == bt.OK, info
    assert info[0]["relres_true"] <= 1e-10
    assert true_relres(d["D"], d["O"], d["b"], x) <= F64_TRUE_RES
    xd = orc.btchol_solve(d["D"], d["O"], d["b"])
    # kappa ~ 1.7e4 times 1e-10, with margin
    assert_close(x, xd, 1e-6, "float32 + refinement against the direct solve")


def test_single_n12_f32_plain():
    """Pure float32 PCG (float64 sums in the dot products, no refinement) on the
    N = 512, n = 12 system (kappa ~ 1.7e4): run until the float32 iteration
    stagnates (recursive residual 1e-8) and meet the float32 bar of 1e-5
    against the float64 direct solve, globally and per block row."""
    d = workload("single_n12")
    P = bt.Params.polycoeff(2, prec="f32")
    x, info, _ = gpu_solve(d["D"], d["O"], d["b"], params=P, tol=1e-8)
    assert info[0]["status"] == bt.OK, info
    xd = orc.btchol_solve(d["D"], d["O"], d["b"])
    print("pure f32: rel", rel(x, xd), "row max", rowmax_rel(x, xd),
          "true relres", true_relres(d["D"], d["O"], d["b"], x))
    assert_close(x, xd, 1e-5, "pure float32 against the direct solve")


@pytest.mark.parametrize("N,n", [(1, 1), (1, 5), (2, 1), (2, 3), (3, 2),
                                 (7, 1), (17, 4), (64, 12), (70, 16),
                                 (40, 24), (24, 32), (12, 48), (6, 64),
                                 (1, 48)])
def test_shapes_and_ragged_tails(N, n):
    """Sizes spanning several elements per thread and ragged tails."""
    d = lqrgen.lqr_instance(N, n, max(1, n // 3), 4242, N * 100 + n)
    _check_f64(d["D"], d["O"], d["b"], bt.Params.polycoeff(2))


@pytest.mark.parametrize("N,n", [(682, 12), (256, 32), (128, 64)])
def test_single_system_at_workgroup_capacity(N, n):
    """The largest single systems one workgroup holds (N n <= 8192 unknowns):
    float64 parity with the oracle and float32 + refinement to 1e-10; one
    block row more is refused by bt_solve (bt_solve_grid takes it)."""
    import torch
    d = lqrgen.lqr_instance(N, n, max(1, n // 3), 4343, N + n, s=0.05)
    _check_f64(d["D"], d["O"], d["b"], bt.Params.polycoeff(2))
    x, info, _ = gpu_solve(d["D"], d["O"], d["b"],
                           params=bt.Params.polycoeff(2, prec="f32_ir"))
    assert info[0]["status"] == bt.OK and info[0]["relres_true"] <= 1e-10
    big = lqrgen.lqr_instance(N + 1, n, max(1, n // 3), 4343, 0, s=0.05)
    assert (N + 1) * n > 8192
    h = bt.Handle(to_dev(big["D"], torch.float64),
                  to_dev(big["O"], torch.float64), None,
                  bt.Params.polycoeff(2))
    bb = to_dev(big["b"].reshape(-1), torch.float64)
    with pytest.raises(bt.BtError):
        h.solve(bb)
    xg, ig = h.solve_grid(bb)
    torch.cuda.synchronize()
    assert bt.infos_to_numpy(ig)[0]["status"] == bt.OK


def test_batch_f64_per_instance_parity():
    B = 24
    data = lqrgen.lqr_batch(B, (1, 40), 5, 2, seed=77)
    P = bt.Params.polycoeff(2)
    x, info, _ = gpu_solve(data["D"], data["O"], data["b"], data["offsets"], P)
    for i, rows, oblk in orc.batch_slices(data["offsets"]):
        xr, ri = orc.pcg(data["D"][rows], data["O"][oblk], data["b"][rows],
                         m=2, alpha=orc.polycoeff(2))
        assert info[i]["status"] == bt.OK
        assert iteration_match(int(info[i]["iters"]), ri), (i, info[i], ri)
        if info[i]["iters"] == ri["iters"]:
            assert_close(x[rows], xr, 1e-10, i)


@pytest.mark.parametrize("n", [16, 24, 48])
def test_batch_f64_larger_blocks(n):
    """Setup kernels of the larger block sizes (wavefront-per-row factors,
    row-wavefront or block F) across instance boundaries, lengths 1..20."""
    data = lqrgen.lqr_batch(12, (1, 20), n, n // 3, seed=500 + n)
    P = bt.Params.polycoeff(2)
    x, info, _ = gpu_solve(data["D"], data["O"], data["b"], data["offsets"], P)
    for i, rows, oblk in orc.batch_slices(data["offsets"]):
        xr, ri = orc.pcg(data["D"][rows], data["O"][oblk], data["b"][rows],
                         m=2, alpha=orc.polycoeff(2))
        assert info[i]["status"] == bt.OK
        assert iteration_match(int(info[i]["iters"]), ri), (i, info[i], ri)
        if info[i]["iters"] == ri["iters"]:
            assert_close(x[rows], xr, 1e-10, i)


def test_batch_f32_refinement_small():
    B = 64
    data = lqrgen.lqr_batch(B, (16, 64), 12, 4, seed=91, record="f32")
    P = bt.Params.polycoeff(2, prec="f32_ir")
    x, info, _ = gpu_solve(data["D"], data["O"], data["b"], data["offsets"], P,
                           record="f32")
    assert np.all(info["status"] == bt.OK), info
    assert np.all(info["relres_true"] <= 1e-10)
    for i, rows, oblk in orc.batch_slices(data["offsets"]):
        if i % 8:
            continue
        xd = orc.btchol_solve(data["D"][rows], data["O"][oblk], data["b"][rows])
        assert true_relres(data["D"][rows], data["O"][oblk], data["b"][rows],
                           x[rows]) <= F64_TRUE_RES
        assert_close(x[rows], xd, 1e-5, i)


@pytest.mark.parametrize("name", ["polycoeff_m2", "jacobi_m2", "stairs_m2",
                                  "equal_m3", "none", "polycoeff_m1"])
def test_precondition_matches_oracle(name):
    import torch
    d = lqrgen.lqr_instance(20, 6, 2, 5, 1)
    P = VARIANTS[name]
    h = bt.Handle(torch.tensor(d["D"], device="cuda"),
                  torch.tensor(d["O"], device="cuda"), None, P)
    r = np.random.default_rng(3).standard_normal((20, 6))
    z = h.precondition(torch.tensor(r.reshape(-1), device="cuda"))
    zr = orc.precond(d["D"], d["O"], r, **oracle_kind(P))
    assert rel(z.cpu().numpy().reshape(20, 6), zr) <= 1e-12


def test_precondition_f32():
    import torch
    d = lqrgen.lqr_instance(20, 6, 2, 5, 1)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    h = bt.Handle(torch.tensor(d["D"], device="cuda", dtype=torch.float32),
                  torch.tensor(d["O"], device="cuda", dtype=torch.float32),
                  None, P)
    r = np.random.default_rng(3).standard_normal((20, 6))
    z = h.precondition(torch.tensor(r.reshape(-1), device="cuda"))
    D32 = d["D"].astype(np.float32).astype(np.float64)
    O32 = d["O"].astype(np.float32).astype(np.float64)
    zr = orc.precond(D32, O32, r, m=2, alpha=orc.polycoeff(2))
    assert rel(z.cpu().numpy().reshape(20, 6), zr) <= 1e-4


# ------------------------------------------------------------- edge cases
def test_zero_rhs_and_single_block():
    d = lqrgen.lqr_instance(1, 4, 2, 1, 0)
    x, info, _ = gpu_solve(d["D"], d["O"], np.zeros((1, 4)),
                           params=bt.Params.polycoeff(2))
    assert info[0]["status"] == bt.OK and info[0]["iters"] == 0
    assert not np.any(x)
    x, info, _ = gpu_solve(d["D"], d["O"], d["b"], params=bt.Params.polycoeff(2))
    assert info[0]["iters"] == 1
    assert rel(x, np.linalg.solve(d["D"][0], d["b"][0])[None]) <= 1e-13


def test_not_spd_block_reported():
    data = lqrgen.lqr_batch(3, 6, 3, 1, seed=3)
    D = data["D"].copy()
    D[6 + 4] = -np.eye(3)          # instance 1, block row 4
    x, info, _ = gpu_solve(D, data["O"], data["b"], data["offsets"],
                           bt.Params.polycoeff(2))
    assert info[1]["status"] == bt.ENOTSPD and info[1]["fail_index"] == 4
    assert info[0]["status"] == bt.OK and info[2]["status"] == bt.OK


def test_iteration_cap_and_nonfinite():
    d = lqrgen.lqr_instance(32, 6, 3, 9, 0)
    x, info, _ = gpu_solve(d["D"], d["O"], d["b"], params=bt.Params(pc="none",
                                                                     m=1),
                           maxit=5)
    assert info[0]["status"] == bt.NOT_CONVERGED and info[0]["iters"] == 5
    xr, ri = orc.pcg(d["D"], d["O"], d["b"], kind=orc.PC_NONE, maxit=5)
    assert rel(x, xr) <= 1e-11
    b = d["b"].copy()
    b[3, 2] = np.nan
    x, info, _ = gpu_solve(d["D"], d["O"], b, params=bt.Params.polycoeff(2))
    assert info[0]["status"] == bt.ENONFINITE


def test_indefinite_system_breaks_down():
    """A with SPD diagonal blocks but indefinite as a whole (upper blocks
    placed untransposed in the LQR recipe, large enough to lose SPD)."""
    D = np.stack([np.eye(1)] * 2)
    O = np.array([[[2.0]]])
    x, info, _ = gpu_solve(D, O, np.array([[1.0], [-1.0]]),
                           params=bt.Params(pc="none", m=1))
    assert info[0]["status"] == bt.EBREAKDOWN


def test_deterministic_repeat():
    d = workload("single_n12")
    x1, i1, _ = gpu_solve(d["D"], d["O"], d["b"], params=bt.Params.polycoeff(2))
    x2, i2, _ = gpu_solve(d["D"], d["O"], d["b"], params=bt.Params.polycoeff(2))
    assert np.array_equal(x1, x2) and i1[0]["iters"] == i2[0]["iters"]


# ---------------------------------------------------------------- adjoint
def test_adjoint_matches_oracle_gradient():
    import torch
    data = lqrgen.lqr_batch(3, (6, 12), 4, 2, seed=12, with_target=True)
    D, O, b, t = data["D"], data["O"], data["b"], data["t"]
    Dt = torch.tensor(D, device="cuda", requires_grad=True)
    Ot = torch.tensor(O, device="cuda", requires_grad=True)
    bt_ = torch.tensor(b, device="cuda", requires_grad=True)
    tt = torch.tensor(t, device="cuda")
    x = bt.bt_solve(Dt, Ot, bt_, data["offsets"], bt.Params.polycoeff(2),
                    tol=1e-13)
    loss = ((x - tt) ** 2).sum()
    loss.backward()
    for i, rows, oblk in orc.batch_slices(data["offsets"]):
        xo = orc.btchol_solve(D[rows], O[oblk], b[rows])
        lam, dD, dO = orc.adjoint(D[rows], O[oblk], xo, 2 * (xo - t[rows]))
        assert rel(bt_.grad[rows].cpu().numpy(), lam) <= 1e-9
        assert rel(Dt.grad[rows].cpu().numpy(), dD) <= 1e-9
        assert rel(Ot.grad[oblk].cpu().numpy(), dO) <= 1e-9


# ------------------------------------------------------ block-gemv counters
def _g(P):
    if P.pc == "none":
        return 3
    return 2 * P.m + 2 if P.a == 0 else 3 * P.m + 3 if P.a == 1 else 5 * P.m + 1


@pytest.mark.parametrize("name", ["polycoeff_m2", "polycoeff_m3", "jacobi_m1",
                                  "stairs_m2", "none"])
def test_gemv_counters_f64(name):
    """bt_info carries the paper's count iters * g_a(m) (Section IV-B) and the
    block products the float64 solve executed: per iteration one application
    of C for A p and the preconditioner's, each two products per row (one on
    the end rows), one triangular product per row for the stopping test
    ||L rhat||, two more transforms and the final float64 residual."""
    d = lqrgen.lqr_instance(40, 6, 2, 8, 3)
    P = VARIANTS[name]
    x, info, _ = gpu_solve(d["D"], d["O"], d["b"], params=P)
    it, N = int(info[0]["iters"]), 40
    assert info[0]["status"] == bt.OK and it > 0
    assert info[0]["gemv_paper"] == it * _g(P)
    if P.pc == "none":
        apc, tri = 0, it + 2 + it   # z = L^T (L r) at each preconditioning
    else:
        apc = (1 if P.a != 0 else 0) + (P.m - 1) * (2 if P.a != 0 else 1)
        tri = it + 2
    want = 2 * (N - 1) * (apc * it + it) + N * tri + (3 * N - 2)
    assert info[0]["gemv_exec"] == want, (info[0]["gemv_exec"], want)


def test_gemv_counters_refinement():
    """The register-resident float32 kernel: the paper's count from the inner
    iterations, and executed products within the bounds of its arrangement
    (four applications of C per inner iteration at m = 2, plus the
    refinement's transforms and residuals)."""
    data = lqrgen.lqr_batch(16, (20, 60), 12, 4, seed=19, record="f32")
    P = bt.Params.polycoeff(2, prec="f32_ir")
    x, info, _ = gpu_solve(data["D"], data["O"], data["b"], data["offsets"], P,
                           record="f32")
    for i, rows, _ in orc.batch_slices(data["offsets"]):
        N = rows.stop - rows.start
        it, outer = int(info[i]["iters"]), int(info[i]["outer"])
        assert info[i]["status"] == bt.OK
        assert info[i]["gemv_paper"] == 9 * it
        lo = 8 * (N - 1) * it
        hi = 8 * (N - 1) * (it + 2 * outer) + 2 * N * outer + \
            (3 * N - 2) * (outer + 1)
        assert lo <= info[i]["gemv_exec"] <= hi, (i, info[i], lo, hi)


# ----------------------------------------- right-hand sides far from unit scale
@pytest.mark.parametrize("scale", [1e-14, 1e18])
@pytest.mark.parametrize("path", ["fast", "generic", "grid"])
def test_refinement_with_scaled_rhs(scale, path):
    """Float32 inner solves see the float64 residual scaled to unit norm, so
    b of any scale converges as b of unit scale does (same iterations) and
    x scales with b."""
    import torch
    data = lqrgen.lqr_batch(1 if path == "grid" else 8, (24, 60), 12, 4,
                            seed=23, record="f32")
    P = bt.Params.polycoeff(2, prec="f32_ir")
    D = to_dev(data["D"], torch.float32)
    O = to_dev(data["O"], torch.float32)
    h = bt.Handle(D, O, data["offsets"], P)
    if path == "generic":
        cfgs = [c for c, nt, s, pr in bt.kernel_configs() if s > 0 and
                pr == bt.F32 and nt * s >= 60 * 12]
        h.set_kernel_config(cfgs[0])
    out = {}
    for sc in (1.0, scale):
        b = to_dev((data["b"] * sc).reshape(-1), torch.float64)
        x, info = h.solve_grid(b) if path == "grid" else h.solve(b)
        torch.cuda.synchronize()
        out[sc] = (x.cpu().numpy().reshape(-1, 12), bt.infos_to_numpy(info))
    x1, i1 = out[1.0]
    xs, is_ = out[scale]
    assert np.all(is_["status"] == bt.OK), is_
    assert np.all(is_["relres_true"] <= 1e-10)
    # the scaled residual rounds differently in float32 (the scale is not a
    # power of two), so the counts may differ by a little
    assert np.all(np.abs(i1["iters"] - is_["iters"]) <=
                  np.maximum(2, i1["iters"] // 10)), (i1, is_)
    for i, rows, oblk in orc.batch_slices(data["offsets"]):
        Di, Oi, bi = data["D"][rows], data["O"][oblk], data["b"][rows] * scale
        assert true_relres(Di, Oi, bi, xs[rows]) <= F64_TRUE_RES
        assert_close(xs[rows], orc.btchol_solve(Di, Oi, bi), 1e-6, i)


def test_autograd_solve_raises_on_failure():
    """bt_solve (the autograd Function) checks every instance's status: a
    non-SPD D_k raises BtError instead of handing x to autograd."""
    import torch
    data = lqrgen.lqr_batch(3, 6, 3, 1, seed=3)
    D = data["D"].copy()
    D[6 + 4] = -np.eye(3)
    Dt = torch.tensor(D, device="cuda", requires_grad=True)
    Ot = torch.tensor(data["O"], device="cuda", requires_grad=True)
    b = torch.tensor(data["b"], device="cuda", requires_grad=True)
    with pytest.raises(bt.BtError) as e:
        bt.bt_solve(Dt, Ot, b, data["offsets"], bt.Params.polycoeff(2))
    assert e.value.code == bt.ENOTSPD
    # unchecked: the infos are the caller's to read
    x = bt.bt_solve(Dt, Ot, b, data["offsets"], bt.Params.polycoeff(2),
                    check=False)
    assert x.shape == b.shape
