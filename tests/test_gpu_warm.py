"""Initial guess (bt_params.warm_start): every solve path starts from the x
passed in. Float64: iteration counts equal the oracle's PCG from the same x0
and solutions agree with its iterate to 1e-10. Float32 + refinement and the
matrix-core path: the float64 residual reaches 1e-10 with fewer iterations
than from zero, and none from the solution itself. b = 0 gives x = 0 whatever
x0 is; the adjoint ignores the setting."""
from dataclasses import replace

import numpy as np
import pytest

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt
from gpu_util import (F64_TRUE_RES, assert_close, iteration_match, oracle_kind,
                      rel, to_dev, true_relres)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bt.load_library()


def handle(D, O, offsets, P, record="f64"):
    import torch
    dt = torch.float64 if record == "f64" else torch.float32
    return bt.Handle(to_dev(D, dt), to_dev(O, dt) if len(O) else None,
                     offsets, P)


def run(h, b, x0, path="solve", tol=1e-10, maxit=None):
    import torch
    n = h.n
    bt_ = to_dev(np.asarray(b).reshape(-1), torch.float64)
    x = to_dev(np.asarray(x0).reshape(-1), torch.float64)
    if path == "grid":
        x, info = h.solve_grid(bt_, tol, maxit, x=x)
    else:
        x, info = h.solve(bt_, tol, maxit, x=x)
    torch.cuda.synchronize()
    return x.cpu().numpy().reshape(-1, n), bt.infos_to_numpy(info)


def starts(d, seed):
    """A start near the solution and a random one."""
    xd = orc.btchol_solve(d["D"], d["O"], d["b"])
    rng = np.random.default_rng(seed)
    return {"near": xd + 1e-4 * np.abs(xd).max() * rng.standard_normal(xd.shape),
            "random": rng.standard_normal(xd.shape)}


VARIANTS = {"polycoeff_m2": bt.Params.polycoeff(2),
            "jacobi_m2": bt.Params.block_jacobi(2),
            "opt_m1": bt.Params(a=1.0, m=1)}


@pytest.mark.parametrize("path", ["solve", "grid"])
@pytest.mark.parametrize("name", sorted(VARIANTS))
@pytest.mark.parametrize("N,n", [(32, 6), (130, 12)])
def test_f64_from_x0_matches_oracle(N, n, name, path):
    d = lqrgen.lqr_instance(N, n, max(1, n // 3), 21, N + n)
    P = replace(VARIANTS[name], warm_start=True)
    h = handle(d["D"], d["O"], None, P)
    for which, x0 in starts(d, N).items():
        x, info = run(h, d["b"], x0, path)
        xr, ri = orc.pcg(d["D"], d["O"], d["b"], tol=1e-10, x0=x0,
                         **oracle_kind(P))
        assert ri["status"] == orc.OK and info[0]["status"] == bt.OK, \
            (which, info)
        assert iteration_match(int(info[0]["iters"]), ri), (which, info, ri)
        if info[0]["iters"] == ri["iters"]:
            assert_close(x, xr, 1e-10, which)
        assert info[0]["relres_true"] <= F64_TRUE_RES
        assert true_relres(d["D"], d["O"], d["b"], x) <= F64_TRUE_RES
    # a cold start needs more iterations than the near one
    _, ri0 = orc.pcg(d["D"], d["O"], d["b"], tol=1e-10, **oracle_kind(P))
    _, rin = orc.pcg(d["D"], d["O"], d["b"], tol=1e-10,
                     x0=starts(d, N)["near"], **oracle_kind(P))
    assert rin["iters"] < ri0["iters"]


def test_f64_batch_from_x0_matches_oracle():
    data = lqrgen.lqr_batch(24, (5, 60), 6, 2, seed=33)
    P = replace(bt.Params.polycoeff(2), warm_start=True)
    h = handle(data["D"], data["O"], data["offsets"], P)
    rng = np.random.default_rng(5)
    x0 = rng.standard_normal(data["b"].shape)
    x, info = run(h, data["b"], x0)
    for i, rows, oblk in orc.batch_slices(data["offsets"]):
        D, O, b = data["D"][rows], data["O"][oblk], data["b"][rows]
        xr, ri = orc.pcg(D, O, b, tol=1e-10, x0=x0[rows], **oracle_kind(P))
        assert info[i]["status"] == bt.OK
        assert iteration_match(int(info[i]["iters"]), ri), (i, info[i], ri)
        if info[i]["iters"] == ri["iters"]:
            assert_close(x[rows], xr, 1e-10, i)
        assert true_relres(D, O, b, x[rows]) <= F64_TRUE_RES


@pytest.mark.parametrize("path", ["fast", "generic", "grid"])
def test_f32_refinement_from_x0(path):
    if path == "grid":
        d = lqrgen.lqr_instance(300, 12, 4, 44, 0)
        data = dict(D=d["D"], O=d["O"], b=d["b"], offsets=None)
    else:
        data = lqrgen.lqr_batch(64, (16, 200), 12, 4, seed=44, record="f32")
    P = bt.Params.polycoeff(2, prec="f32_ir", inner_tol=1e-5)
    Pw = replace(P, warm_start=True)
    cold = handle(data["D"], data["O"], data["offsets"], P, "f32")
    warm = handle(data["D"], data["O"], data["offsets"], Pw, "f32")
    if path == "generic":
        generic = [c[0] for c in bt.kernel_configs()
                   if c[3] == bt.F32 and c[2] > 0 and c[1] * c[2] >= 200 * 12]
        for h in (cold, warm):
            h.set_kernel_config(generic[0])
    elif path == "fast":
        assert warm.kernel_config() in [c[0] for c in bt.kernel_configs()
                                        if c[2] == 0]
    pth = "grid" if path == "grid" else "solve"
    b = data["b"]
    x1, i1 = run(cold, b, np.zeros_like(b), pth)
    assert np.all(i1["status"] == bt.OK)
    # the next right-hand side of a sequence, started from the last solution
    rng = np.random.default_rng(6)
    b2 = b + 1e-3 * rng.standard_normal(b.shape)
    xc, ic = run(cold, b2, np.zeros_like(b), pth)
    xw, iw = run(warm, b2, x1, pth)
    assert np.all(iw["status"] == bt.OK) and np.all(iw["relres_true"] <= 1e-10)
    assert iw["iters"].sum() < ic["iters"].sum()
    assert rel(xw, xc) <= 1e-8
    # from the solution itself: no iteration, no refinement step
    x3, i3 = run(warm, b2, xw, pth)
    assert np.all(i3["status"] == bt.OK) and np.all(i3["iters"] == 0)
    assert np.all(i3["outer"] == 0)
    assert np.array_equal(x3, xw)


@pytest.mark.parametrize("path", ["solve", "grid"])
@pytest.mark.parametrize("prec", ["f64", "f32_ir"])
def test_zero_rhs_gives_zero_from_any_start(path, prec):
    d = lqrgen.lqr_instance(40, 6, 2, 8, 1)
    P = replace(bt.Params.polycoeff(2, prec=prec), warm_start=True)
    h = handle(d["D"], d["O"], None, P)
    x, info = run(h, np.zeros_like(d["b"]), np.ones_like(d["b"]), path)
    assert info[0]["status"] == bt.OK and info[0]["iters"] == 0
    assert not np.any(x)


def test_warm_start_needs_an_initial_guess():
    import torch
    d = lqrgen.lqr_instance(20, 6, 2, 8, 1)
    h = handle(d["D"], d["O"], None,
               replace(bt.Params.polycoeff(2), warm_start=True))
    with pytest.raises(ValueError):
        h.solve(to_dev(d["b"].reshape(-1), torch.float64))


def test_adjoint_ignores_warm_start():
    import torch
    d = lqrgen.lqr_instance(50, 6, 2, 9, 2)
    P = bt.Params.polycoeff(2)
    g = to_dev(np.random.default_rng(1).standard_normal(d["b"].size),
               torch.float64)
    x = to_dev(orc.btchol_solve(d["D"], d["O"], d["b"]).reshape(-1),
               torch.float64)
    out = []
    for p in (P, replace(P, warm_start=True)):
        h = handle(d["D"], d["O"], None, p)
        lam, dD, dO, info = h.adjoint(x, g)
        torch.cuda.synchronize()
        out.append((lam.cpu().numpy(), dD.cpu().numpy(),
                    bt.infos_to_numpy(info)[0]["iters"]))
    assert out[0][2] == out[1][2]
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_mrhs_from_x0():
    import torch
    d = lqrgen.lqr_instance(256, 16, 5, 10, 0, nrhs=64)
    P = bt.Params.polycoeff(2, prec="bf16x2_ir", inner_tol=1e-4)
    D32 = to_dev(d["D"], torch.float32)
    O32 = to_dev(d["O"], torch.float32)
    Dr = d["D"].astype(np.float32).astype(np.float64)
    Or = d["O"].astype(np.float32).astype(np.float64)
    B = to_dev(d["b"], torch.float64)
    cold = bt.Handle(D32, O32, None, P)
    warm = bt.Handle(D32, O32, None, replace(P, warm_start=True))
    X1, i1 = cold.solve_mrhs(B)
    torch.cuda.synchronize()
    i1 = bt.infos_to_numpy(i1)
    assert np.all(i1["status"] == bt.OK)
    # perturbed right-hand sides, started from the last solutions
    rng = np.random.default_rng(3)
    B2 = to_dev(d["b"] + 1e-3 * rng.standard_normal(d["b"].shape),
                torch.float64)
    Xc, ic = cold.solve_mrhs(B2)
    Xw, iw = warm.solve_mrhs(B2, X=X1.clone())
    torch.cuda.synchronize()
    ic, iw = bt.infos_to_numpy(ic), bt.infos_to_numpy(iw)
    assert np.all(iw["status"] == bt.OK) and np.all(iw["relres_true"] <= 1e-10)
    assert iw["iters"].sum() < ic["iters"].sum()
    Xw = Xw.cpu().numpy()
    B2h = B2.cpu().numpy()
    for c in range(0, 64, 9):
        xd = orc.btchol_solve(Dr, Or, B2h[:, :, c])
        assert rel(Xw[:, :, c], xd) <= 1e-8, c
    # zero columns give zero whatever the start
    B3 = B2.clone()
    B3[:, :, 5] = 0.0
    X3, i3 = warm.solve_mrhs(B3, X=torch.ones_like(B3))
    torch.cuda.synchronize()
    assert not torch.any(X3[:, :, 5]).item()
    assert bt.infos_to_numpy(i3)[5]["status"] == bt.OK
