"""The Section V experiment runner (paper_2503_15269_amd.fig2) on a small
sample: every setting converges, the footnote identity of Section III-E
(optimal weights at order m = block Jacobi at order 2m) shows up as equal
spectra and equal iteration counts, and the gemv accounting follows g_a(m)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def res():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_15269_amd import fig2
    return fig2.run(matrices=3, rhs=6, eig_matrices=2)


def row(res, fam, m):
    return [r for r in res["rows"] if r["family"] == fam and r["m"] == m][0]


def test_all_settings_converge(res):
    assert len(res["rows"]) == 5 * 4 - 1
    assert all(r["converged"] for r in res["rows"])


@pytest.mark.parametrize("m", [1, 2])
def test_optimal_m_equals_block_jacobi_2m(res, m):
    o, j = row(res, "Optimal", m), row(res, "Block Jacobi", 2 * m)
    assert abs(o["iters_mean"] - j["iters_mean"]) <= 0.5
    for key in ("lam_min", "lam_max", "cond"):
        assert o[key] == pytest.approx(j[key], rel=1e-7), key


def test_gemv_accounting(res):
    from paper_2503_15269_amd.fig2 import gemv_per_iteration
    for r in res["rows"]:
        assert r["gemv_mean"] == pytest.approx(
            r["iters_mean"] * gemv_per_iteration(r["a"], r["m"]))
    assert gemv_per_iteration(0.0, 2) == 6
    assert gemv_per_iteration(1.0, 2) == 9
    assert gemv_per_iteration(0.5, 2) == 11


def test_optimal_spectrum_inside_unit_interval(res):
    # Theorem 3.5: the eigenvalues of opt M_m^{-1} A lie in (0, 1]
    for m in (1, 2, 3, 4):
        r = row(res, "Optimal", m)
        assert r["lam_min"] > 0 and r["lam_max"] <= 1 + 1e-9
