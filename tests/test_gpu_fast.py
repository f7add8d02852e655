"""The register-resident bin kernel (block sizes 12 and 24, float32 inner PCG
with float64 refinement, optimal weights) against the oracle and against the
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


# largest horizon a bin of the register-resident kernel holds, per block size
BIN_ROWS = {12: 256, 24: 128}


def batch(n, B, horizons, seed, record="f32"):
    """Seeded LQR batch with nu = n / 3; horizons (lo, hi), hi capped at the
    bin capacity for block size n."""
    lo, hi = horizons
    hi = min(hi, BIN_ROWS[n])
    return lqrgen.lqr_batch(B, (min(lo, hi), hi), n, n // 3, seed=seed,
                            record=record)


def fast_indices():
    """Configuration index per variant of the register-resident kernel."""
    return [c[0] for c in bt.kernel_configs() if c[2] == 0]


# (block size, variant): 3, 6 or 12 entries per lane for n = 12, 6 for n = 24
CASES = [(12, 0), (12, 1), (12, 2), (24, 1)]
CASE_IDS = ["n12-ept3", "n12-ept6", "n12-ept12", "n24-ept6"]
case_param = pytest.mark.parametrize("n,v", CASES, ids=CASE_IDS)


def default_variant(n):
    return fast_indices()[0 if n == 12 else 1]


def run(data, params, record="f32", cfg=None, tol=1e-10, maxit=None):
    import torch
    dt = torch.float32 if record == "f32" else torch.float64
    h = bt.Handle(to_dev(data["D"], dt), to_dev(data["O"], dt),
                  data["offsets"], params)
    if cfg is not None:
        h.set_kernel_config(cfg)
    x, info = h.solve(to_dev(data["b"].reshape(-1), torch.float64), tol, maxit)
    torch.cuda.synchronize()
    n = data["D"].shape[1]
    return x.cpu().numpy().reshape(-1, n), bt.infos_to_numpy(info), h


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


@pytest.mark.parametrize("n", [12, 24])
def test_fast_kernel_is_selected(n):
    data = batch(n, 8, (16, 40), seed=1)
    _, _, h = run(data, bt.Params.polycoeff(2, prec="f32_ir"))
    assert h.kernel_config() == default_variant(n)
    # variants that do not apply to the block size are refused
    for v, idx in enumerate(fast_indices()):
        if (n, v) not in CASES:
            with pytest.raises(bt.BtError):
                h.set_kernel_config(idx)


@case_param
@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_fast_polycoeff_orders(m, n, v):
    data = batch(n, 48, (16, 256), seed=100 + m)
    x, info, h = run(data, bt.Params.polycoeff(m, prec="f32_ir"),
                     cfg=fast_indices()[v])
    assert h.kernel_config() == fast_indices()[v]
    check_against_oracle(data, x, info, every=4)


@case_param
def test_fast_vs_generic_same_batch(n, v):
    data = batch(n, 40, (16, 256), seed=7)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    xf, inf_f, hf = run(data, P, cfg=fast_indices()[v])
    generic = [c[0] for c in bt.kernel_configs()
               if c[3] == bt.F32 and c[2] > 0 and
               c[1] * c[2] >= BIN_ROWS[n] * n][0]
    xg, inf_g, hg = run(data, P, cfg=generic)
    check_against_oracle(data, xf, inf_f, every=3)
    check_against_oracle(data, xg, inf_g, every=3)
    for i, rows, _ in orc.batch_slices(data["offsets"]):
        assert rel(xf[rows], xg[rows]) <= 1e-6
    # the fast kernel refuses systems longer than its bins
    over = lqrgen.lqr_batch(2, BIN_ROWS[n] + 1, n, n // 3, seed=8,
                            record="f32")
    _, inf_o, ho = run(over, P)
    assert ho.kernel_config() not in fast_indices()
    assert np.all(inf_o["status"] == bt.OK)
    with pytest.raises(bt.BtError):
        ho.set_kernel_config(fast_indices()[v])


@case_param
def test_fast_many_systems_per_bin(n, v):
    """A batch long enough to need more than one round of bins keeps many
    systems in each bin (the capacity is lowered only as far as the rounds
    allow); a small batch of the same systems spreads over more bins. Both
    solve every system to the tolerance."""
    P = bt.Params.polycoeff(2, prec="f32_ir")
    cfg = fast_indices()[v]
    big = batch(n, 6000, (1, 12), seed=31)
    x, info, _ = run(big, P, cfg=cfg)
    check_against_oracle(big, x, info, every=97)
    small = {k: big[k] for k in ("D", "O", "b")}
    B = 40
    small["offsets"] = big["offsets"][:B + 1]
    R = int(small["offsets"][-1])
    small["D"], small["b"] = big["D"][:R], big["b"][:R]
    small["O"] = big["O"][:R - B]
    xs, infs, _ = run(small, P, cfg=cfg)
    check_against_oracle(small, xs, infs)
    # a system's segment partials meet in a tree fixed by their slots in
    # the bin, so the two packings may round differently: both reach the
    # 1e-10 residual and agree to the conditioning of these short horizons
    assert rel(xs, x[:R]) <= 1e-7


@case_param
def test_fast_packs_tiny_and_mixed_systems(n, v):
    """Bins holding many short systems next to long ones (ragged tails,
    horizons 1..20, and 1 up to the bin capacity)."""
    short = batch(n, 60, (1, 20), seed=21)
    cfg = fast_indices()[v]
    x, info, _ = run(short, bt.Params.polycoeff(2, prec="f32_ir"), cfg=cfg)
    check_against_oracle(short, x, info)
    mixed = batch(n, 30, (1, 256), seed=22)
    x, info, _ = run(mixed, bt.Params.polycoeff(2, prec="f32_ir"), cfg=cfg)
    check_against_oracle(mixed, x, info)


@case_param
def test_fast_f64_record(n, v):
    data = batch(n, 24, (16, 128), seed=5, record="f64")
    x, info, _ = run(data, bt.Params.polycoeff(2, prec="f32_ir"), record="f64",
                     cfg=fast_indices()[v])
    check_against_oracle(data, x, info)


@case_param
def test_fast_failures_and_zero_rhs(n, v):
    data = batch(n, 6, (20, 40), seed=9)
    D = data["D"].copy()
    r0 = int(data["offsets"][2])
    D[r0 + 5] = -np.eye(n)                       # system 2, row 5
    b = data["b"].copy()
    b[int(data["offsets"][3]):int(data["offsets"][4])] = 0.0   # system 3
    b[int(data["offsets"][4]) + 1, 3] = np.inf   # system 4
    d2 = dict(data, D=D, b=b)
    x, info, _ = run(d2, bt.Params.polycoeff(2, prec="f32_ir"),
                     cfg=fast_indices()[v])
    assert info[2]["status"] == bt.ENOTSPD and info[2]["fail_index"] == 5
    assert info[3]["status"] == bt.OK and info[3]["iters"] == 0
    assert info[4]["status"] == bt.ENONFINITE
    for i in (0, 1, 5):
        assert info[i]["status"] == bt.OK and info[i]["relres_true"] <= 1e-10
    rows3 = slice(int(data["offsets"][3]), int(data["offsets"][4]))
    assert not np.any(x[rows3])


@case_param
def test_fast_iteration_cap(n, v):
    data = batch(n, 4, (100, 120), seed=3)
    x, info, _ = run(data, bt.Params.polycoeff(2, prec="f32_ir"), maxit=7,
                     cfg=fast_indices()[v])
    assert np.all(info["status"] == bt.NOT_CONVERGED)
    assert np.all(info["iters"] <= 7)


@case_param
def test_fast_deterministic(n, v):
    data = batch(n, 32, (16, 256), seed=11)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    x1, i1, _ = run(data, P, cfg=fast_indices()[v])
    x2, i2, _ = run(data, P, cfg=fast_indices()[v])
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


def test_autotune_order_picks_the_fastest_converging_m(tmp_path, monkeypatch):
    import torch
    from paper_2503_15269_amd import autotune
    monkeypatch.setenv("BTPCG_TUNE_CACHE", str(tmp_path / "tune.json"))
    data = lqrgen.lqr_batch(32, (16, 200), 12, 4, seed=45, record="f32")
    D = to_dev(data["D"], torch.float32)
    O = to_dev(data["O"], torch.float32)
    b = to_dev(data["b"].reshape(-1), torch.float64)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    res = autotune.tune_order(D, O, data["offsets"], b, P, 1e-10,
                              orders=(1, 2, 3), reps=1, inner_tols=(3e-6,))
    times = {m: t for m, t in res["orders"].items() if t is not None}
    assert set(times) == {1, 2, 3}
    m = res["params"].m
    assert res["ms"] == min(times.values()) == times[m]
    assert res["params"].alpha[m - 1] == (7.0 if m > 1 else 1.0)
    h = bt.Handle(D, O, data["offsets"], res["params"])
    h.set_kernel_config(res["kernel_config"])
    x, info = h.solve(b, 1e-10)
    torch.cuda.synchronize()
    inf = bt.infos_to_numpy(info)
    assert np.all(inf["status"] == bt.OK) and np.all(inf["relres_true"] <= 1e-10)


def test_factors_for_other_kernels_formed_on_first_use():
    """A handle set up for the register-resident kernel forms the Cholesky
    factors L (which only the other kernels read) when a solve, a
    preconditioner application or a refactor first needs them; in-place
    changes of D are picked up."""
    import torch
    data = batch(12, 10, (16, 200), seed=31)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    Dt = to_dev(data["D"], torch.float32)
    Ot = to_dev(data["O"], torch.float32)
    b = to_dev(data["b"].reshape(-1), torch.float64)
    h = bt.Handle(Dt, Ot, data["offsets"], P)
    assert h.kernel_config() == fast_indices()[0]
    generic = [c[0] for c in bt.kernel_configs()
               if c[3] == bt.F32 and c[2] > 0 and c[1] * c[2] >= 200 * 12][0]

    def solve_check(dat):
        x, info = h.solve(b, 1e-10)
        torch.cuda.synchronize()
        check_against_oracle(dat, x.cpu().numpy().reshape(-1, 12),
                             bt.infos_to_numpy(info), every=2)
        return x

    solve_check(data)                      # fast kernel, no L
    z = h.precondition(b)                  # generic kernel: forms L
    assert torch.isfinite(z).all()
    h.set_kernel_config(generic)
    solve_check(data)
    # change D in place: refactor (generic config: L and F as well)
    Dt.mul_(2.0)                           # exact in float32
    d2 = dict(data, D=data["D"] * 2.0)
    h.refactor()
    solve_check(d2)
    h.set_kernel_config(fast_indices()[0])
    solve_check(d2)
    # and back to the generic kernel after a refactor made for the fast one
    Dt.mul_(2.0)
    d3 = dict(data, D=data["D"] * 4.0)
    h.refactor()
    h.set_kernel_config(generic)
    solve_check(d3)


@pytest.mark.parametrize("which", ["fast", "generic"])
def test_graph_replays_match_eager(which):
    """refactor + solve captured into one HIP graph: every replay (with other
    GPU work in between) reproduces the eager result bit for bit, and picks
    up new contents of the input buffers (b scaled by 2 scales x exactly)."""
    import torch
    data = batch(12, 24, (16, 200), seed=41)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    D = to_dev(data["D"], torch.float32)
    O = to_dev(data["O"], torch.float32)
    b = to_dev(data["b"].reshape(-1), torch.float64)
    h = bt.Handle(D, O, data["offsets"], P)
    if which == "generic":
        h.set_kernel_config([c[0] for c in bt.kernel_configs()
                             if c[3] == bt.F32 and c[2] > 0 and
                             c[1] * c[2] >= 200 * 12][0])
    else:
        assert h.kernel_config() in fast_indices()
    x = torch.empty_like(b)
    info = torch.empty((len(data["offsets"]) - 1) * bt.INFO_DTYPE.itemsize,
                       dtype=torch.uint8, device="cuda")
    h.refactor()
    h.solve(b, 1e-10, x=x, info=info)
    torch.cuda.synchronize()
    x_ref, info_ref = x.clone(), info.clone()
    assert np.all(bt.infos_to_numpy(info)["status"] == bt.OK)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        h.refactor()
        h.solve(b, 1e-10, x=x, info=info)
    for rep in range(3):
        x.zero_()
        info.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()   # other work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(x, x_ref), rep
        assert torch.equal(info, info_ref), rep
    b.mul_(2.0)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(x, 2.0 * x_ref)
    i2, i1 = bt.infos_to_numpy(info), bt.infos_to_numpy(info_ref)
    assert np.array_equal(i2["iters"], i1["iters"])


@pytest.mark.parametrize("n", [12, 24])
def test_graph_replay_after_an_eager_full_setup(n):
    """A captured refactor + solve of the register-resident kernel keeps
    reading its own packed L^{-1} after an eager call on the same handle
    switched it to the full factors (the preconditioner runs on the generic
    kernel and sets up L and the full L^{-1} first): every replay reproduces
    the eager result."""
    import torch
    data = batch(n, 24, (16, 120), seed=71)
    P = bt.Params.polycoeff(2, prec="f32_ir")
    D = to_dev(data["D"], torch.float32)
    O = to_dev(data["O"], torch.float32)
    b = to_dev(data["b"].reshape(-1), torch.float64)
    h = bt.Handle(D, O, data["offsets"], P)
    assert h.kernel_config() in fast_indices()
    x = torch.empty_like(b)
    info = torch.empty((len(data["offsets"]) - 1) * bt.INFO_DTYPE.itemsize,
                       dtype=torch.uint8, device="cuda")
    h.refactor()
    h.solve(b, 1e-10, x=x, info=info)
    torch.cuda.synchronize()
    x_ref, info_ref = x.clone(), info.clone()
    assert np.all(bt.infos_to_numpy(info)["status"] == bt.OK)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        h.refactor()
        h.solve(b, 1e-10, x=x, info=info)
    z = h.precondition(b)          # eager: full setup of the same handle
    torch.cuda.synchronize()
    assert torch.isfinite(z).all()
    for rep in range(3):
        x.zero_()
        info.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref), rep
        assert torch.equal(info, info_ref), rep
        h.precondition(b)          # and again between replays
    # an eager solve after all this agrees as well
    x2, info2 = h.solve(b, 1e-10)
    torch.cuda.synchronize()
    assert torch.equal(x2, x_ref)
