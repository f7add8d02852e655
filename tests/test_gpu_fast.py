"""The register-resident bin kernel (block size 12, float32 inner PCG with
float64 refinement, optimal weights) against the oracle and against the
generic kernel on the same inputs."""
import numpy as np
import pytest

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt
from gpu_util import rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bt.load_library()


def fast_index():
    return [c[0] for c in bt.kernel_configs() if c[2] == 0][0]


def run(data, params, record="f32", cfg=None, tol=1e-10, maxit=None):
    import torch
    dt = torch.float32 if record == "f32" else torch.float64
    h = bt.Handle(to_dev(data["D"], dt), to_dev(data["O"], dt),
                  data["offsets"], params)
    if cfg is not None:
        h.set_kernel_config(cfg)
    x, info = h.solve(to_dev(data["b"].reshape(-1), torch.float64), tol, maxit)
    torch.cuda.synchronize()
    return x.cpu().numpy().reshape(-1, 12), bt.infos_to_numpy(info), h


def check_against_oracle(data, x, info, every=1, tol=1e-10):
    assert np.all(info["status"] == bt.OK), np.unique(info["status"])
    assert np.all(info["relres_true"] <= tol)
    for i, rows, oblk in orc.batch_slices(data["offsets"]):
        if i % every:
            continue
        D, O, b = data["D"][rows], data["O"][oblk], data["b"][rows]
        r = b - orc.spmv(D, O, x[rows])
        assert np.linalg.norm(r) <= 1.01 * tol * np.linalg.norm(b), i
        xd = orc.btchol_solve(D, O, b)
        assert rel(x[rows], xd) <= 1e-5, (i, rel(x[rows], xd))


def test_fast_kernel_is_selected():
    data = lqrgen.lqr_batch(8, (16, 40), 12, 4, seed=1, record="f32")
    _, _, h = run(data, bt.Params.polycoeff(2, prec="f32_ir"))
    assert h.kernel_config() == fast_index()


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_fast_polycoeff_orders(m):
    data = lqrgen.lqr_batch(48, (16, 256), 12, 4, seed=100 + m, record="f32")
    x, info, _ = run(data, bt.Params.polycoeff(m, prec="f32_ir"))
    check_against_oracle(data, x, info, every=4)


def test_fast_vs_generic_same_batch():
    data = lqrgen.lqr_batch(40, (16, 256), 12, 4, seed=7, record="f32")
    P = bt.Params.polycoeff(2, prec="f32_ir")
    xf, inf_f, hf = run(data, P)
    assert hf.kernel_config() == fast_index()
    generic = [c[0] for c in bt.kernel_configs()
               if c[3] == bt.F32 and c[2] > 0 and c[1] * c[2] >= 256 * 12][0]
    xg, inf_g, hg = run(data, P, cfg=generic)
    check_against_oracle(data, xf, inf_f, every=3)
    check_against_oracle(data, xg, inf_g, every=3)
    for i, rows, _ in orc.batch_slices(data["offsets"]):
        assert rel(xf[rows], xg[rows]) <= 1e-6


def test_fast_packs_tiny_and_mixed_systems():
    """Bins holding many short systems next to long ones (ragged tails,
    horizons 1..20 plus a few of 200..256)."""
    short = lqrgen.lqr_batch(60, (1, 20), 12, 4, seed=21, record="f32")
    x, info, _ = run(short, bt.Params.polycoeff(2, prec="f32_ir"))
    check_against_oracle(short, x, info)
    mixed = lqrgen.lqr_batch(30, (1, 256), 12, 4, seed=22, record="f32")
    x, info, _ = run(mixed, bt.Params.polycoeff(2, prec="f32_ir"))
    check_against_oracle(mixed, x, info)


def test_fast_f64_record():
    data = lqrgen.lqr_batch(24, (16, 128), 12, 4, seed=5, record="f64")
    x, info, _ = run(data, bt.Params.polycoeff(2, prec="f32_ir"), record="f64")
    check_against_oracle(data, x, info)


def test_fast_failures_and_zero_rhs():
    data = lqrgen.lqr_batch(6, (20, 40), 12, 4, seed=9, record="f32")
    D = data["D"].copy()
    r0 = int(data["offsets"][2])
    D[r0 + 5] = -np.eye(12)                      # system 2, row 5
    b = data["b"].copy()
    b[int(data["offsets"][3]):int(data["offsets"][4])] = 0.0   # system 3
    b[int(data["offsets"][4]) + 1, 3] = np.inf   # system 4
    d2 = dict(data, D=D, b=b)
    x, info, _ = run(d2, bt.Params.polycoeff(2, prec="f32_ir"))
    assert info[2]["status"] == bt.ENOTSPD and info[2]["fail_index"] == 5
    assert info[3]["status"] == bt.OK and info[3]["iters"] == 0
    assert info[4]["status"] == bt.ENONFINITE
    for i in (0, 1, 5):
        assert info[i]["status"] == bt.OK and info[i]["relres_true"] <= 1e-10
    rows3 = slice(int(data["offsets"][3]), int(data["offsets"][4]))
    assert not np.any(x[rows3])


def test_fast_iteration_cap():
    data = lqrgen.lqr_batch(4, (100, 120), 12, 4, seed=3, record="f32")
    x, info, _ = run(data, bt.Params.polycoeff(2, prec="f32_ir"), maxit=7)
    assert np.all(info["status"] == bt.NOT_CONVERGED)
    assert np.all(info["iters"] <= 7)


def test_fast_deterministic():
    data = lqrgen.lqr_batch(32, (16, 256), 12, 4, seed=11, record="f32")
    P = bt.Params.polycoeff(2, prec="f32_ir")
    x1, i1, _ = run(data, P)
    x2, i2, _ = run(data, P)
    assert np.array_equal(x1, x2)
    assert np.array_equal(i1["iters"], i2["iters"])


def test_autotune_picks_a_converging_config(tmp_path, monkeypatch):
    import torch
    from paper_2503_15269_amd import autotune
    monkeypatch.setenv("BTPCG_TUNE_CACHE", str(tmp_path / "tune.json"))
    data = lqrgen.lqr_batch(32, (16, 200), 12, 4, seed=44, record="f32")
    D = to_dev(data["D"], torch.float32)
    O = to_dev(data["O"], torch.float32)
    b = to_dev(data["b"].reshape(-1), torch.float64)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    res = autotune.tune(D, O, data["offsets"], b, P, 1e-10, reps=1,
                        inner_tols=(1e-4, 3e-6))
    assert res["ms"] > 0 and not res["cached"]
    assert res["params"].inner_tol in (1e-4, 3e-6)
    again = autotune.tune(D, O, data["offsets"], b, P, 1e-10, reps=1,
                          inner_tols=(1e-4, 3e-6))
    assert again["cached"] and again["kernel_config"] == res["kernel_config"]
    h = bt.Handle(D, O, data["offsets"], res["params"])
    h.set_kernel_config(res["kernel_config"])
    x, info = h.solve(b, 1e-10)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)
    assert np.all(inf["status"] == bt.OK) and np.all(inf["relres_true"] <= 1e-10)
