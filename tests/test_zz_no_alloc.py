"""bt_solve_grid_noalloc: the grid-wide single-system solve with the
library's static scratch instead of a workspace argument, through the C-ABI.
Its output must equal bt_solve_grid's (same kernels, same arithmetic:
bitwise) and the oracle's PCG iterate (float64: equal iteration count,
1e-10), on two calls in a row, the second with a smaller system, so that
what the first call left in the shared array cannot leak into the second."""
import numpy as np
import pytest

import lqrgen
import oracle as orc
import paper_2503_15269_amd as bt
from gpu_util import (F64_TRUE_RES, assert_close, iteration_match,
                      oracle_kind, to_dev, true_relres)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(oracle_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bt.load_library()


def _both(d, P, record):
    import torch
    dt = torch.float64 if record == "f64" else torch.float32
    h = bt.Handle(to_dev(d["D"], dt), to_dev(d["O"], dt), None, P)
    b = to_dev(d["b"].reshape(-1), torch.float64)
    x0, i0 = h.solve_grid(b)
    x1 = torch.full_like(b, float("nan"))
    info = torch.zeros(bt.INFO_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    x1, i1 = h.solve_grid_noalloc(b, x=x1, info=info)
    torch.cuda.synchronize()
    n = d["D"].shape[1]
    return (x0.cpu().numpy().reshape(-1, n), bt.infos_to_numpy(i0)[0],
            x1.cpu().numpy().reshape(-1, n), bt.infos_to_numpy(i1)[0])


@pytest.mark.parametrize("prec", ["f64", "f32_ir"])
def test_noalloc_matches_grid_solve_twice(prec):
    P = bt.Params.polycoeff(2, prec=prec)
    record = "f64" if prec == "f64" else "f32"
    for N, seed in ((512, 41), (100, 42)):   # second call: smaller system
        d = lqrgen.lqr_instance(N, 12, 4, seed, 0)
        if record == "f32":
            d["D"] = d["D"].astype(np.float32).astype(np.float64)
            d["O"] = d["O"].astype(np.float32).astype(np.float64)
        xg, ig, xs, is_ = _both(d, P, record)
        print(f"N={N} {prec}: iters {is_['iters']} (grid {ig['iters']}), "
              f"relres_true {is_['relres_true']:.2e}")
        assert is_["status"] == bt.OK, is_
        assert np.array_equal(xs, xg), N          # same kernels: bitwise
        assert is_["iters"] == ig["iters"] and is_["outer"] == ig["outer"]
        assert is_["gemv_exec"] == ig["gemv_exec"]
        assert true_relres(d["D"], d["O"], d["b"], xs) <= F64_TRUE_RES
        if prec == "f64":
            xr, ri = orc.pcg(d["D"], d["O"], d["b"], tol=1e-10,
                             **oracle_kind(P))
            assert iteration_match(int(is_["iters"]), ri), (is_, ri)
            if is_["iters"] == ri["iters"]:
                assert_close(xs, xr, 1e-10, N)
        else:
            assert_close(xs, orc.btchol_solve(d["D"], d["O"], d["b"]), 1e-6, N)


def test_noalloc_refuses_a_system_above_its_scratch():
    import torch
    # float64 grid scratch is about 64 bytes per unknown: 11000 x 12 unknowns
    # need more than the 8 MiB the library holds
    N, n = 11000, 12
    d = lqrgen.lqr_instance(N, n, 4, 43, 0)
    h = bt.Handle(to_dev(d["D"], torch.float64), to_dev(d["O"], torch.float64),
                  None, bt.Params.polycoeff(2))
    need = bt.load_library().bt_grid_workspace_bytes(h._h)
    assert need > (8 << 20)
    b = to_dev(d["b"].reshape(-1), torch.float64)
    with pytest.raises(bt.BtError) as e:
        h.solve_grid_noalloc(b)
    assert e.value.code == bt.ENOSPACE
