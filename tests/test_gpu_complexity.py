"""The direct-against-iterative sweep (paper_2503_15269_amd.complexity) on a
small sample: every method succeeds, the direct and PCG solutions agree, and
the report carries the fields the comparison of Section IV-C needs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def res():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15269_amd import complexity
    return complexity.run(single_N=(16, 256), batch_N=(32,), B=64, reps=2)


def test_every_method_succeeds(res):
    for r in res["single"] + res["batch"]:
        assert r["direct_ok"], r
        assert r["pcg_f64_ok"] and r["pcg_f32_ir_ok"], r


def test_direct_and_pcg_agree(res):
    # PCG stops at a relative residual of 1e-10; these systems have
    # condition numbers below 1e4
    for r in res["single"] + res["batch"]:
        assert r["pcg_f64_rel_diff"] <= 1e-6, r
        assert r["pcg_f32_ir_rel_diff"] <= 1e-6, r


def test_report_fields(res):
    for r in res["single"]:
        for k in ("direct_ms", "pcg_f64_ms", "pcg_f32_ir_ms",
                  "pcg_f64_setup_ms"):
            assert np.isfinite(r[k]) and r[k] > 0, (k, r)
        assert r["pcg_f64_iters"] > 0
        # both sizes fit one workgroup: the faster PCG path is reported
        for prec in ("f64", "f32_ir"):
            wg = r[f"pcg_{prec}_workgroup_ms"]
            assert wg is not None and wg > 0
            assert r[f"pcg_{prec}_ms"] == min(wg, r[f"pcg_{prec}_grid_ms"])
    assert set(res["summary"]) == {"single", "batch"}
    from paper_2503_15269_amd import complexity
    assert "| N |" in complexity.markdown(res)
