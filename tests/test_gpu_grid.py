"""The grid-wide single-system solve (bt_solve_grid) against the oracle.

Float64: iteration counts equal the oracle's PCG (same rule as the other
parity tests) and solutions agree with it to 1e-10; the single-workgroup
path (bt_solve) gives the same count. Float32 + refinement: the float64
residual of the record reaches 1e-10 and the error against the oracle's
block Cholesky solve stays within the float32 bound. Sizes span several
workgroups with a ragged last one, a system above the single-workgroup
capacity, and the degenerate cases.
"""
import numpy as np
import pytest

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt
from gpu_util import (F64_TRUE_RES, assert_close, iteration_match, oracle_kind,
                      rel, to_dev, true_relres, workload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bt.load_library()


def grid_solve(D, O, b, params, tol=1e-10, maxit=None, record="f64"):
    import torch
    dt = torch.float64 if record == "f64" else torch.float32
    n = D.shape[1]
    h = bt.Handle(to_dev(D, dt), to_dev(O, dt) if len(O) else None, None,
                  params)
    x, info = h.solve_grid(to_dev(np.asarray(b).reshape(-1), torch.float64),
                           tol, maxit)
    torch.cuda.synchronize()
    return x.cpu().numpy().reshape(-1, n), bt.infos_to_numpy(info), h


VARIANTS = {
    "polycoeff_m2": bt.Params.polycoeff(2),
    "polycoeff_m3": bt.Params.polycoeff(3),
    "opt_m1": bt.Params(a=1.0, m=1),
    "jacobi_m2": bt.Params.block_jacobi(2),
    "stairs_m2": bt.Params(a=0.5, m=2),
    "none": bt.Params(pc="none", m=1),
}

# (N, n): one workgroup, several with a ragged last one, many
SHAPES = [(7, 6), (45, 12), (130, 5), (300, 12), (60, 24)]


@pytest.mark.parametrize("N,n", SHAPES)
@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_grid_f64_matches_oracle(N, n, name):
    P = VARIANTS[name]
    d = lqrgen.lqr_instance(N, n, max(1, n // 3), 11, N + n)
    x, info, _ = grid_solve(d["D"], d["O"], d["b"], P)
    xr, ri = orc.pcg(d["D"], d["O"], d["b"], tol=1e-10, maxit=10 * N * n,
                     **oracle_kind(P))
    assert ri["status"] == orc.OK
    assert info[0]["status"] == bt.OK, info
    # plain CG (no preconditioner) runs past the dimension of the system and
    # its count depends on the rounding order of the dot products (here the
    # grid's per-workgroup partial sums): 3% slack there; every
    # preconditioner of the paper must match exactly
    slack = max(2, 3 * ri["iters"] // 100) if P.pc == "none" else 0
    assert iteration_match(int(info[0]["iters"]), ri, slack=slack), (info, ri)
    if info[0]["iters"] == ri["iters"]:
        assert_close(x, xr, 1e-10, "against the oracle's PCG iterate")
    else:  # both converged iterates agree to the conditioning bound
        assert_close(x, orc.btchol_solve(d["D"], d["O"], d["b"]), 1e-6,
                     "against the direct solve")
    assert info[0]["relres"] <= 1e-10
    assert info[0]["relres_true"] <= F64_TRUE_RES
    assert true_relres(d["D"], d["O"], d["b"], x) <= F64_TRUE_RES


@pytest.mark.parametrize("name", ["polycoeff_m2", "jacobi_m2"])
def test_grid_same_count_as_single_workgroup_path(name):
    import torch
    d = workload("single_n12")
    P = VARIANTS[name]
    x, info, h = grid_solve(d["D"], d["O"], d["b"], P)
    x1, i1 = h.solve(to_dev(d["b"].reshape(-1), torch.float64), 1e-10)
    i1 = bt.infos_to_numpy(i1)
    assert info[0]["iters"] == i1[0]["iters"]
    assert rel(x, x1.cpu().numpy().reshape(x.shape)) <= 1e-11


@pytest.mark.parametrize("record", ["f32", "f64"])
def test_grid_f32_refinement(record):
    d = workload("single_n12")
    D, O = d["D"], d["O"]
    if record == "f32":
        D = D.astype(np.float32).astype(np.float64)
        O = O.astype(np.float32).astype(np.float64)
    P = bt.Params.polycoeff(2, prec="f32_ir", inner_tol=1e-4)
    x, info, _ = grid_solve(D, O, d["b"], P, record=record)
    assert info[0]["status"] == bt.OK, info
    assert info[0]["relres_true"] <= 1e-10
    assert info[0]["outer"] >= 2
    assert true_relres(D, O, d["b"], x) <= F64_TRUE_RES
    xd = orc.btchol_solve(D, O, d["b"])
    assert_close(x, xd, 1e-5, "against the direct solve")


def test_grid_above_single_workgroup_capacity():
    # 2048 x 12 = 24576 unknowns: bt_solve cannot hold it, bt_solve_grid can
    import torch
    d = lqrgen.lqr_instance(2048, 12, 4, 3, 0)
    P = bt.Params.polycoeff(2)
    x, info, h = grid_solve(d["D"], d["O"], d["b"], P)
    assert info[0]["status"] == bt.OK, info
    assert info[0]["relres_true"] <= F64_TRUE_RES
    assert true_relres(d["D"], d["O"], d["b"], x) <= F64_TRUE_RES
    xd = orc.btchol_solve(d["D"], d["O"], d["b"])
    assert_close(x, xd, 1e-8, "against the direct solve")
    with pytest.raises(bt.BtError):
        h.solve(to_dev(d["b"].reshape(-1), torch.float64), 1e-10)


@pytest.mark.parametrize("prec", ["f64", "f32_ir"])
def test_grid_n48_blocks_read_from_memory(prec):
    # n = 48: the window's blocks do not fit the LDS staging area, so C reads
    # them from memory; float32 record for the refinement case
    d = lqrgen.lqr_instance(600, 48, 16, 9, 0, s=0.05)
    D, O = d["D"], d["O"]
    record = "f32" if prec == "f32_ir" else "f64"
    if record == "f32":
        D = D.astype(np.float32).astype(np.float64)
        O = O.astype(np.float32).astype(np.float64)
    P = bt.Params.polycoeff(2, prec=prec)
    x, info, _ = grid_solve(D, O, d["b"], P, record=record)
    assert info[0]["status"] == bt.OK, info
    assert info[0]["relres_true"] <= (1e-10 if prec == "f32_ir"
                                      else F64_TRUE_RES)
    assert true_relres(D, O, d["b"], x) <= F64_TRUE_RES
    xd = orc.btchol_solve(D, O, d["b"])
    assert rel(x, xd) <= 1e-6, rel(x, xd)
    if prec == "f64":
        xr, ri = orc.pcg(D, O, d["b"], tol=1e-10, **oracle_kind(P))
        assert iteration_match(int(info[0]["iters"]), ri), (info, ri)


def test_grid_zero_rhs_and_iteration_cap():
    d = lqrgen.lqr_instance(45, 12, 4, 5, 1)
    P = bt.Params.polycoeff(2)
    x, info, _ = grid_solve(d["D"], d["O"], np.zeros_like(d["b"]), P)
    assert info[0]["status"] == bt.OK and info[0]["iters"] == 0
    assert not np.any(x)
    x, info, _ = grid_solve(d["D"], d["O"], d["b"], P, maxit=3)
    assert info[0]["status"] == bt.NOT_CONVERGED and info[0]["iters"] == 3
    # the iterate after 3 steps equals the oracle's
    xr, ri = orc.pcg(d["D"], d["O"], d["b"], tol=1e-30, maxit=3,
                     **oracle_kind(P))
    assert ri["iters"] == 3
    assert rel(x, xr) <= 1e-10


@pytest.mark.parametrize("N", [1, 2, 5])
def test_grid_tiny_horizons(N):
    d = lqrgen.lqr_instance(N, 6, 2, 12, N)
    P = bt.Params.polycoeff(2)
    x, info, _ = grid_solve(d["D"], d["O"], d["b"], P)
    xr, ri = orc.pcg(d["D"], d["O"], d["b"], tol=1e-10, **oracle_kind(P))
    assert info[0]["status"] == bt.OK, info
    assert iteration_match(int(info[0]["iters"]), ri), (info, ri)
    assert rel(x, orc.btchol_solve(d["D"], d["O"], d["b"])) <= 1e-9


def test_grid_non_finite_rhs():
    d = lqrgen.lqr_instance(45, 6, 2, 13, 0)
    b = d["b"].copy()
    b[7, 2] = np.nan
    for prec in ("f64", "f32_ir"):
        _, info, _ = grid_solve(d["D"], d["O"], b,
                                bt.Params.polycoeff(2, prec=prec))
        assert info[0]["status"] == bt.ENONFINITE, (prec, info)


def test_grid_not_spd_block():
    d = lqrgen.lqr_instance(45, 6, 2, 6, 2)
    D = d["D"].copy()
    D[20] = -np.eye(6)
    x, info, _ = grid_solve(D, d["O"], d["b"], bt.Params.polycoeff(2))
    assert info[0]["status"] == bt.ENOTSPD
    assert info[0]["fail_index"] == 20


def test_grid_argument_checks():
    import torch
    d = workload("batch_ragged_n12", instances=3)
    h = bt.Handle(to_dev(d["D"], torch.float64), to_dev(d["O"], torch.float64),
                  d["offsets"], bt.Params.polycoeff(2))
    with pytest.raises(bt.BtError):  # more than one system
        h.solve_grid(to_dev(d["b"].reshape(-1), torch.float64))


@pytest.mark.parametrize("prec", ["f64", "f32_ir"])
def test_grid_repeated_solves_and_iteration_cap(prec):
    """Repeated solves on one handle give the same result bit for bit (the
    barrier state and every partial are reset or rewritten per solve), and
    an iteration cap stops the iteration exactly."""
    import torch
    d = lqrgen.lqr_instance(300, 12, 4, 17, 3)
    P = bt.Params.polycoeff(2, prec=prec)
    h = bt.Handle(to_dev(d["D"], torch.float64), to_dev(d["O"], torch.float64),
                  None, P)
    b = to_dev(d["b"].reshape(-1), torch.float64)
    out = []
    for _ in range(3):
        x, info = h.solve_grid(b)
        torch.cuda.synchronize()
        out.append((x.cpu().numpy(), bt.infos_to_numpy(info)[0]))
    assert out[0][1]["status"] == bt.OK
    for x, inf in out[1:]:
        assert np.array_equal(x, out[0][0])
        assert inf["iters"] == out[0][1]["iters"]
    x, info = h.solve_grid(b, maxit=3)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)[0]
    assert inf["status"] == bt.NOT_CONVERGED and inf["iters"] == 3
    if prec == "f64":
        xr, ri = orc.pcg(d["D"], d["O"], d["b"], tol=1e-30, maxit=3,
                         **oracle_kind(P))
        assert rel(x.cpu().numpy().reshape(xr.shape), xr) <= 1e-10


@pytest.mark.parametrize("N,n", [(300, 12), (40000, 6), (2000, 48),
                                 (8192, 12), (32768, 12)])
def test_grid_more_windows_than_resident_workgroups(N, n):
    """Long systems: windows of 4 to 64 rows (N = 8192, n = 12: 32 rows, one
    window per CU; N = 32768: 64 rows, two per workgroup), and systems with
    more row windows than one pass of the grid holds, where each workgroup
    loops over several windows; float64 counts equal the oracle's where the
    oracle finishes quickly, otherwise the true residual and the error
    against the direct solve."""
    d = lqrgen.lqr_instance(N, n, max(1, n // 3), 29, N, s=0.05)
    P = bt.Params.polycoeff(2)
    x, info, _ = grid_solve(d["D"], d["O"], d["b"], P)
    assert info[0]["status"] == bt.OK, info
    assert true_relres(d["D"], d["O"], d["b"], x) <= F64_TRUE_RES
    assert_close(x, orc.btchol_solve(d["D"], d["O"], d["b"]), 1e-7,
                 "against the direct solve")
    if N * n <= 4000:
        xr, ri = orc.pcg(d["D"], d["O"], d["b"], tol=1e-10, **oracle_kind(P))
        assert iteration_match(int(info[0]["iters"]), ri), (info, ri)


def test_grid_deep_window_above_64kb_of_lds():
    """n = 48 at m = 7 (a = 1): a window carries 14 halo rows on each side,
    so a workgroup needs more than 64 KB of LDS and the launch raises the
    kernel's limit (within the 160 KB a workgroup has beside the kernel's
    static LDS); the true residual and the error against the direct solve."""
    N, n, m = 600, 48, 7
    rb = max(4, min(16, N // 64))
    depth = 1 + 2 * (m - 1) + 1
    assert 256 * 8 + 5 * (rb + 2 * depth) * n * 8 > 64 * 1024
    d = lqrgen.lqr_instance(N, n, 16, 41, 0, s=0.05)
    x, info, _ = grid_solve(d["D"], d["O"], d["b"], bt.Params(a=1.0, m=m))
    assert info[0]["status"] == bt.OK, info
    assert true_relres(d["D"], d["O"], d["b"], x) <= F64_TRUE_RES
    assert_close(x, orc.btchol_solve(d["D"], d["O"], d["b"]), 1e-7,
                 "against the direct solve")


def test_grid_barrier_gives_up_and_the_handle_recovers():
    """A barrier wait limit of zero makes a grid barrier give up: every
    workgroup returns, the solve reports ETIMEOUT, and the next solve with
    the default limit on the same handle is correct."""
    import torch
    d = lqrgen.lqr_instance(512, 12, 4, 31, 0)
    P = bt.Params.polycoeff(2)
    h = bt.Handle(to_dev(d["D"], torch.float64), to_dev(d["O"], torch.float64),
                  None, P)
    b = to_dev(d["b"].reshape(-1), torch.float64)
    h.set_grid_wait(0.0)
    x, info = h.solve_grid(b)
    torch.cuda.synchronize()
    assert bt.infos_to_numpy(info)[0]["status"] == bt.ETIMEOUT
    h.set_grid_wait(2.0)
    x, info = h.solve_grid(b)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)[0]
    xr, ri = orc.pcg(d["D"], d["O"], d["b"], tol=1e-10, **oracle_kind(P))
    assert inf["status"] == bt.OK and iteration_match(int(inf["iters"]), ri)
    if inf["iters"] == ri["iters"]:
        assert_close(x.cpu().numpy().reshape(-1, 12), xr, 1e-10, "after")
