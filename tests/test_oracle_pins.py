"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every check compares the oracle with something that is not the oracle: dense
matrices assembled from the paper's definitions and handled by numpy's LAPACK
routines, closed forms, spectral theorems, the paper's tables (fixtures under
tests/golden/) and finite differences.
"""
import os

import numpy as np
import pytest

import lqrgen
import oracle as orc
from dense import G_H_ab, M_inv, dense_A, op_matrix, random_bt, splittings

EPS = np.finfo(np.float64).eps
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def lqr(N, nx, nu, seed=11, inst=0, s=0.1):
    d = lqrgen.lqr_instance(N, nx, nu, seed, inst, s=s)
    return d["D"], d["O"], d["b"]


def f_pm(a, lam):
    """f_{a+-}(lambda) = a lambda +- (1-a) sqrt(lambda), Section III-B."""
    s = np.sqrt(lam)
    return a * lam + (1 - a) * s, a * lam - (1 - a) * s


def nonzero_eigs_BlCl(D, O):
    S = splittings(D, O)
    ev = np.linalg.eigvals(np.linalg.solve(S["Bl"], S["Cl"]))
    return ev


# ---------------------------------------------------------------- inputs
@pytest.mark.parametrize("N,nx,nu", [(1, 3, 2), (2, 3, 1), (5, 4, 2),
                                     (8, 6, 3)])
def test_generator_is_the_kkt_schur_complement(N, nx, nu):
    """Section V: A = C H^-1 C^T of the LQR QP; SPD."""
    d = lqrgen.lqr_instance(N, nx, nu, 7, 3, keep_dynamics=True)
    C, H = lqrgen.kkt_dense(d["A"], d["Bm"], d["q"], d["r"])
    S = C @ np.linalg.solve(H, C.T)
    A = dense_A(d["D"], d["O"])
    assert np.abs(S - A).max() <= 1e-12 * np.abs(S).max()
    assert np.linalg.eigvalsh(A).min() > 0


def test_generator_is_seeded_and_records_round():
    a = lqrgen.lqr_batch(3, (4, 9), 3, 2, seed=5, record="f32")
    b = lqrgen.lqr_batch(3, (4, 9), 3, 2, seed=5, record="f32")
    for k in ("D", "O", "b", "offsets"):
        assert np.array_equal(a[k], b[k])
    assert np.array_equal(a["D"], a["D"].astype(np.float32).astype(np.float64))
    assert a["offsets"][-1] == a["D"].shape[0]
    assert a["O"].shape[0] == a["D"].shape[0] - 3
    assert np.all((a["horizons"] >= 4) & (a["horizons"] <= 9))


# ------------------------------------------------------ direct solver
@pytest.mark.parametrize("N,n", [(1, 1), (1, 4), (2, 1), (3, 2), (7, 3),
                                 (32, 6)])
def test_block_cholesky_matches_dense_solve(N, n):
    D, O, b = lqr(N, n, max(1, n // 2))
    A = dense_A(D, O)
    x = orc.btchol_solve(D, O, b).reshape(-1)
    xd = np.linalg.solve(A, b.reshape(-1))
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(x - xd) <= 1e2 * EPS * kappa * np.linalg.norm(xd)


def test_block_cholesky_multi_rhs_and_generic():
    D, O = random_bt(9, 3, seed=2)
    rng = np.random.default_rng(1)
    B = rng.standard_normal((9, 3, 4))
    X = orc.btchol_solve(D, O, B)
    A = dense_A(D, O)
    for j in range(4):
        assert np.allclose(A @ X[:, :, j].reshape(-1), B[:, :, j].reshape(-1),
                           atol=1e-12)


def test_block_cholesky_rejects_indefinite():
    D = np.stack([np.eye(2)] * 3)
    O = np.stack([2.0 * np.eye(2)] * 2)          # eigenvalues 1 +- 2 sqrt 2
    with pytest.raises(np.linalg.LinAlgError):
        orc.btchol_solve(D, O, np.ones((3, 2)))


def test_spmv_matches_dense():
    D, O, _ = lqr(6, 4, 2)
    x = np.random.default_rng(0).standard_normal((6, 4))
    assert np.allclose(orc.spmv(D, O, x).reshape(-1),
                       dense_A(D, O) @ x.reshape(-1), rtol=1e-14, atol=1e-13)


# ------------------------------------------- preconditioner: closed form
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 8])
@pytest.mark.parametrize("n", [1, 3])
def test_closed_form_Gopt_Hopt_match_definitions(N, n):
    """Section IV-A closed form == eq. (def-GH-ab-multi-splitting) at (1,-1),
    and H_opt == I - G_opt A (Lemma 3.1 proof)."""
    D, O = random_bt(N, n, seed=100 + N * 10 + n)
    blk = orc.setup_opt(D, O)
    for k in range(N):
        assert np.allclose(blk["Dinv"][k], np.linalg.inv(D[k]), rtol=1e-12,
                           atol=1e-12)
    G = op_matrix(lambda r: orc.apply_Gopt(blk, r), N, n)
    H = op_matrix(lambda v: orc.apply_Hopt(blk, v), N, n)
    Gd, Hd = G_H_ab(D, O, 1.0, -1.0)
    A = dense_A(D, O)
    assert np.allclose(G, Gd, rtol=1e-11, atol=1e-11)
    assert np.allclose(H, Hd, rtol=1e-11, atol=1e-11)
    assert np.allclose(H, np.eye(N * n) - Gd @ A, atol=1e-10)
    # H_opt: super/sub-diagonal blocks vanish (Section III-D); G_opt symmetric
    for k in range(N - 1):
        assert np.abs(H[k * n:(k + 1) * n, (k + 1) * n:(k + 2) * n]).max() < 1e-12
        assert np.abs(H[(k + 1) * n:(k + 2) * n, k * n:(k + 1) * n]).max() < 1e-12
    assert np.allclose(G, G.T, atol=1e-13)


AB = [(1.0, -1.0), (0.5, 0.0), (0.0, 1.0), (0.25, 0.5), (1 / 3, 1 / 3),
      (0.75, -0.5)]


@pytest.mark.parametrize("a,b", AB)
def test_splitting_form_matches_definition(a, b):
    N, n = 5, 2
    D, O = random_bt(N, n, seed=41)
    G = op_matrix(lambda r: orc.apply_Gab(D, O, a, b, r), N, n)
    H = op_matrix(lambda v: orc.apply_Hab(D, O, a, b, v), N, n)
    Gd, Hd = G_H_ab(D, O, a, b)
    assert np.allclose(G, Gd, rtol=1e-11, atol=1e-11)
    assert np.allclose(H, Hd, rtol=1e-11, atol=1e-11)
    # Lemma 3.1 proof: G_ab A + H_ab = I on the admissible line 2a+b = 1
    assert np.allclose(G @ dense_A(D, O) + H, np.eye(N * n), atol=1e-10)


def test_splitting_pictures_are_splittings():
    """A = B_d - C_d = B_l - C_l = B_r - C_r (Section II-C)."""
    D, O = random_bt(6, 2, seed=3)
    A = dense_A(D, O)
    S = splittings(D, O)
    for B, C in (("Bd", "Cd"), ("Bl", "Cl"), ("Br", "Cr")):
        assert np.array_equal(S[B] - S[C], A)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", [orc.PC_OPT, orc.PC_SPLIT])
def test_precond_matches_dense_polynomial(m, kind):
    """Eq. (Mminv-polynomial-coefficients) with alpha_{m-1} = 7."""
    N, n = 6, 2
    D, O = random_bt(N, n, seed=8)
    alpha = [1.0] * m
    if m > 1:
        alpha[m - 1] = 7.0
    Mi = op_matrix(lambda r: orc.precond(D, O, r, kind=kind, a=1.0, b=-1.0,
                                         m=m, alpha=alpha), N, n)
    Gd, Hd = G_H_ab(D, O, 1.0, -1.0)
    assert np.allclose(Mi, M_inv(Gd, Hd, m, alpha), rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_footnote_identity_opt_m_equals_jacobi_2m(m):
    """Footnote to Theorem 3.6: M_m^{-1}(1,-1) = M_{2m}^{-1}(0,1)."""
    D, O, b = lqr(9, 4, 2)
    r = np.random.default_rng(m).standard_normal((9, 4))
    z1 = orc.precond(D, O, r, kind=orc.PC_OPT, m=m)
    z2 = orc.precond(D, O, r, kind=orc.PC_SPLIT, a=0.0, b=1.0, m=2 * m)
    assert np.allclose(z1, z2, rtol=1e-11, atol=1e-11 * np.abs(z1).max())


def test_precond_none_is_identity():
    D, O, b = lqr(4, 3, 1)
    assert np.array_equal(orc.precond(D, O, b, kind=orc.PC_NONE), b)


# -------------------------------------------------------- spectra
@pytest.mark.parametrize("N,n", [(4, 2), (5, 2), (6, 3), (7, 1)])
def test_spectrum_of_BlinvCl(N, n):
    """Lemma 3.3 and the proof of Theorem 3.6: floor(N/2) n nonzero
    eigenvalues, all real and in (0,1)."""
    D, O = random_bt(N, n, seed=N * 7 + n)
    ev = nonzero_eigs_BlCl(D, O)
    nz = ev[np.abs(ev) > 1e-9]
    assert len(nz) == (N // 2) * n
    assert np.abs(nz.imag).max() < 1e-9
    assert np.all((nz.real > 0) & (nz.real < 1))


@pytest.mark.parametrize("a,b", AB)
@pytest.mark.parametrize("N", [4, 5])
def test_eigs_of_Hab_GabA_MabinvA_from_lambda(a, b, N):
    """Lemmas 3.1 and 3.2: each nonzero lambda of B_l^-1 C_l gives the pair
    f_{a+-}(lambda) of H_ab, 1 - f of G_ab A, 1 - f^m of M_m^-1 A.
    For odd N the remaining n eigenvalues of M_m^-1 A equal one."""
    n, m = 2, 3
    D, O = random_bt(N, n, seed=500 + N)
    ev = nonzero_eigs_BlCl(D, O)
    lam = np.sort(ev[np.abs(ev) > 1e-9].real)
    fp, fm = f_pm(a, lam)
    pred_H = np.concatenate([fp, fm])
    H = op_matrix(lambda v: orc.apply_Hab(D, O, a, b, v), N, n)
    G = op_matrix(lambda r: orc.apply_Gab(D, O, a, b, r), N, n)
    A = dense_A(D, O)
    eH = np.linalg.eigvals(H)
    eGA = np.linalg.eigvals(G @ A)
    Mi = op_matrix(lambda r: orc.precond(D, O, r, kind=orc.PC_SPLIT, a=a,
                                         b=b, m=m), N, n)
    Ms = 0.5 * (Mi + Mi.T)
    R = np.linalg.cholesky(Ms)
    eM = np.linalg.eigvalsh(R.T @ A @ R)

    def covered(pred, got):
        got = np.sort_complex(got.astype(complex))
        used = np.zeros(len(got), bool)
        for p in np.sort(pred):
            d = np.abs(got - p)
            d[used] = np.inf
            j = int(np.argmin(d))
            if d[j] > 1e-7:
                return False
            used[j] = True
        return True

    assert covered(pred_H, eH)
    assert covered(1 - pred_H, eGA)
    assert covered(1 - pred_H ** m, eM)
    if N % 2 == 1:
        assert np.sum(np.abs(eM - 1.0) < 1e-9) >= n
    else:
        assert len(pred_H) == N * n


def _load_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_spectrum_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                N, n, mat, z, d, p, o = line.split()
                rows.append((int(N), int(n), mat, int(z), int(d), int(p),
                             int(o)))
    return rows


@pytest.mark.parametrize("row", _load_table1(), ids=lambda r: f"{r[0]}x{r[1]}-{r[2]}")
def test_table1_counts(row):
    """Table I: exact zeros, distinct values in (0,1), pairing, exact ones."""
    N, n, mat, zeros, distinct, paired, ones = row
    D, O = random_bt(N, n, seed=1000 + N * 10 + n)
    A = dense_A(D, O)
    S = splittings(D, O)
    blk = orc.setup_opt(D, O)
    G = op_matrix(lambda r: orc.apply_Gopt(blk, r), N, n)
    H = op_matrix(lambda v: orc.apply_Hopt(blk, v), N, n)
    if mat == "BlinvCl":
        M = np.linalg.solve(S["Bl"], S["Cl"])
    elif mat == "Hopt":
        M = H
    elif mat == "GoptA":
        M = G @ A
    elif mat == "HoptGoptA":
        M = H @ G @ A
    elif mat == "IpHoptGoptA":
        M = (np.eye(N * n) + H) @ G @ A
    else:
        m = int(mat.split("_m")[1])
        M = op_matrix(lambda r: orc.precond(D, O, r, kind=orc.PC_OPT, m=m),
                      N, n) @ A
    ev = np.linalg.eigvals(M)
    assert np.abs(ev.imag).max() < 1e-6
    ev = np.sort(ev.real)
    tol = 1e-11     # "exact" zeros/ones; genuine values sit well away (Z17)
    nz = int(np.sum(np.abs(ev) < tol))
    no = int(np.sum(np.abs(ev - 1) < tol))
    inner = ev[(ev > tol) & (ev < 1 - tol)]
    # cluster the interior values
    clusters = []
    for v in inner:
        if clusters and abs(v - clusters[-1][-1]) < 1e-7:
            clusters[-1].append(v)
        else:
            clusters.append([v])
    assert nz == zeros
    assert no == ones
    assert len(clusters) == distinct
    sizes = {len(c) for c in clusters}
    assert sizes == ({2} if paired else {1})


def _load_table2():
    rows = []
    with open(os.path.join(GOLDEN, "table2_intervals.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(float(t) for t in line.split()))
    return rows


@pytest.mark.parametrize("row", _load_table2(), ids=lambda r: f"a={r[0]:.3f}")
def test_table2_ranges_and_oracle_spectra(row):
    """Table II / Lemma 3.4: range of f_{a-} on (0,1) and the interval
    I_{G_ab A}; the oracle's G_ab A and H_ab spectra fall inside."""
    a, inf_fm, sup_fm, upper = row
    lam = np.concatenate([np.geomspace(1e-16, 1e-3, 2000),
                          np.linspace(1e-3, 1 - 1e-12, 400001)])
    _, fm = f_pm(a, lam)
    assert abs(fm.min() - inf_fm) < 1e-6
    assert abs(fm.max() - sup_fm) < 1e-6
    b = 1 - 2 * a
    N, n = 6, 2
    D, O, _ = lqr(N, n, 1, seed=77)
    G = op_matrix(lambda r: orc.apply_Gab(D, O, a, b, r), N, n)
    H = op_matrix(lambda v: orc.apply_Hab(D, O, a, b, v), N, n)
    eGA = np.linalg.eigvals(G @ dense_A(D, O)).real
    eH = np.linalg.eigvals(H).real
    assert eGA.min() > 0 and eGA.max() <= upper + 1e-9
    assert eH.min() >= inf_fm - 1e-9 and eH.max() < 1


@pytest.mark.parametrize("a", [0.0, 0.2, 1 / 3, 0.5, 0.8, 1.0])
def test_theorem_spd_on_Cg(a):
    """Theorem 3.5: on C_g, G_ab is SPD, rho(H_ab) < 1, M_m^-1 SPD."""
    b = 1 - 2 * a
    N, n = 7, 2
    D, O, _ = lqr(N, n, 1, seed=5)
    G = op_matrix(lambda r: orc.apply_Gab(D, O, a, b, r), N, n)
    assert np.allclose(G, G.T, atol=1e-12)
    np.linalg.cholesky(G)
    H = op_matrix(lambda v: orc.apply_Hab(D, O, a, b, v), N, n)
    assert np.abs(np.linalg.eigvals(H)).max() < 1
    for m in (1, 2, 3, 4):
        Mi = op_matrix(lambda r: orc.precond(D, O, r, kind=orc.PC_SPLIT, a=a,
                                             b=b, m=m), N, n)
        assert np.allclose(Mi, Mi.T, atol=1e-10 * np.abs(Mi).max())
        np.linalg.cholesky(0.5 * (Mi + Mi.T))


def test_opt_has_largest_smallest_eigenvalue():
    """Proof of Theorem 3.6: lambda_min(M_m^-1 A) is largest at a = 1."""
    N, n, m = 6, 2, 2
    D, O, _ = lqr(N, n, 1, seed=9)
    A = dense_A(D, O)

    def lmin(a):
        Mi = op_matrix(lambda r: orc.precond(D, O, r, kind=orc.PC_SPLIT, a=a,
                                             b=1 - 2 * a, m=m), N, n)
        R = np.linalg.cholesky(0.5 * (Mi + Mi.T))
        return np.linalg.eigvalsh(R.T @ A @ R).min()

    best = lmin(1.0)
    for a in (0.0, 0.25, 0.5, 0.75, 0.9):
        assert best >= lmin(a) - 1e-12


# ------------------------------------------- distinct eigenvalues / PCG
@pytest.mark.parametrize("N,n", [(2, 1), (3, 1), (4, 1), (5, 1), (4, 2),
                                 (6, 3), (7, 2)])
def test_distinct_eigs_and_finite_termination(N, n):
    """Theorems 3.6/3.7 count d_{Nna}; PCG ends in at most d iterations
    (Section IV-C, finite termination of CG in exact arithmetic)."""
    D, O = random_bt(N, n, seed=3000 + 10 * N + n, off=0.5)
    A = dense_A(D, O)
    b = np.random.default_rng(N).standard_normal((N, n))
    for a, kind, m, alpha in ((1.0, orc.PC_OPT, 1, None),
                              (1.0, orc.PC_OPT, 2, (1, 7)),
                              (0.0, orc.PC_SPLIT, 1, None),
                              (0.5, orc.PC_SPLIT, 1, None)):
        d = orc.distinct_eigenvalue_bound(N, n, a)
        Mi = op_matrix(lambda r: orc.precond(D, O, r, kind=kind, a=a,
                                             b=1 - 2 * a, m=m, alpha=alpha),
                       N, n)
        R = np.linalg.cholesky(0.5 * (Mi + Mi.T))
        ev = np.sort(np.linalg.eigvalsh(R.T @ A @ R))
        distinct = 1 + int(np.sum(np.diff(ev) > 1e-7))
        assert distinct == d, (a, m, distinct, d)
        x, info = orc.pcg(D, O, b, kind=kind, a=a, b=1 - 2 * a, m=m,
                          alpha=alpha, tol=1e-12, maxit=5 * N * n)
        assert info["status"] == orc.OK
        assert info["iters"] <= d
        assert np.allclose(A @ x.reshape(-1), b.reshape(-1), atol=1e-9)


def test_N2_n1_closed_form_one_iteration():
    """N=2, n=1: G_opt = (1 - lambda) A^-1 with lambda = o^2/(d1 d2), so
    G_opt A = (1-lambda) I and PCG stops after one iteration."""
    D = np.array([[[2.0]], [[3.0]]])
    O = np.array([[[1.5]]])
    lam = 1.5 ** 2 / (2.0 * 3.0)
    A = dense_A(D, O)
    blk = orc.setup_opt(D, O)
    G = op_matrix(lambda r: orc.apply_Gopt(blk, r), 2, 1)
    assert np.allclose(G, (1 - lam) * np.linalg.inv(A), rtol=1e-14)
    x, info = orc.pcg(D, O, np.array([[1.0], [-2.0]]), m=1, tol=1e-14)
    assert info["iters"] == 1 and info["status"] == orc.OK
    assert np.allclose(x.reshape(-1), np.linalg.solve(A, [1.0, -2.0]),
                       rtol=1e-14)


def test_N1_is_direct():
    """N = 1: H = 0 and G = D^-1 = A^-1; one iteration for every m."""
    D, O, b = lqr(1, 5, 2)
    for m in (1, 2, 4):
        x, info = orc.pcg(D, O, b, m=m, tol=1e-14)
        assert info["iters"] == 1
        assert np.allclose(x, np.linalg.solve(D[0], b[0])[None], rtol=1e-13)


def test_pcg_solution_and_monotone_in_m():
    """PCG converges to A^-1 b at the workload-1 shape; larger m never needs
    more iterations (Remark 3.1); opt m=1,2 match Jacobi m=2,4 (footnote)."""
    D, O, b = lqr(32, 6, 3, seed=lqrgen.workload_seed(0))
    A = dense_A(D, O)
    xd = np.linalg.solve(A, b.reshape(-1))
    kappa = np.linalg.cond(A)
    its = []
    for m in (1, 2, 3, 4):
        x, info = orc.pcg(D, O, b, m=m, alpha=None, tol=1e-10)
        assert info["status"] == orc.OK
        r = np.linalg.norm(b.reshape(-1) - A @ x.reshape(-1))
        assert r <= 1.01e-10 * np.linalg.norm(b) * 10
        assert np.linalg.norm(x.reshape(-1) - xd) <= 10 * kappa * 1e-10 * \
            np.linalg.norm(xd)
        its.append(info["iters"])
    assert all(its[i] >= its[i + 1] for i in range(3))
    for m in (1, 2):
        x1, i1 = orc.pcg(D, O, b, kind=orc.PC_OPT, m=m, alpha=None)
        x2, i2 = orc.pcg(D, O, b, kind=orc.PC_SPLIT, a=0.0, b=1.0, m=2 * m,
                         alpha=None)
        assert i1["iters"] == i2["iters"]
        assert np.allclose(x1, x2, rtol=1e-8, atol=1e-10)


def test_pcg_gemv_accounting():
    """g_a(m) of Section IV-B."""
    for m in range(1, 6):
        assert orc.gemv_per_iteration(orc.PC_OPT, 1.0, m) == 3 * m + 3
        assert orc.gemv_per_iteration(orc.PC_SPLIT, 0.0, m) == 2 * m + 2
        assert orc.gemv_per_iteration(orc.PC_SPLIT, 0.5, m) == 5 * m + 1


def test_pcg_failure_modes():
    # indefinite A: no preconditioner, p^T A p < 0 at the first step
    D = np.array([[[1.0]], [[1.0]]])
    O = np.array([[[2.0]]])
    _, info = orc.pcg(D, O, np.array([[1.0], [-1.0]]), kind=orc.PC_NONE)
    assert info["status"] == orc.EBREAKDOWN
    # a non-SPD diagonal block
    D2, O2, b2 = lqr(4, 3, 1)
    D2 = D2.copy()
    D2[2] = -np.eye(3)
    _, info = orc.pcg(D2, O2, b2)
    assert info["status"] == orc.ENOTSPD
    # iteration cap
    D3, O3, b3 = lqr(16, 4, 2)
    _, info = orc.pcg(D3, O3, b3, kind=orc.PC_NONE, tol=1e-14, maxit=3)
    assert info["status"] == orc.NOT_CONVERGED and info["iters"] == 3
    # b = 0: zero iterations
    x, info = orc.pcg(D3, O3, np.zeros_like(b3))
    assert info["iters"] == 0 and info["status"] == orc.OK
    assert not np.any(x)


# ---------------------------------------------------------------- adjoint
def test_adjoint_matches_dense_gradient():
    """dL/dA = -lambda x^T restricted to the block-tridiagonal pattern."""
    N, n = 5, 3
    D, O, b = lqr(N, n, 2)
    x = orc.btchol_solve(D, O, b)
    g = np.random.default_rng(4).standard_normal((N, n))
    lam, dD, dO = orc.adjoint(D, O, x, g)
    A = dense_A(D, O)
    lam_d = np.linalg.solve(A, g.reshape(-1))
    assert np.allclose(lam.reshape(-1), lam_d, rtol=1e-10, atol=1e-12)
    GA = -np.outer(lam_d, x.reshape(-1))
    for k in range(N):
        assert np.allclose(dD[k], GA[k * n:(k + 1) * n, k * n:(k + 1) * n])
    for k in range(N - 1):
        up = GA[k * n:(k + 1) * n, (k + 1) * n:(k + 2) * n]
        lo = GA[(k + 1) * n:(k + 2) * n, k * n:(k + 1) * n]
        assert np.allclose(dO[k], up + lo.T)


def test_adjoint_matches_finite_differences():
    """Central differences (h = 1e-6) of L = sum ||x_k - t_k||^2 through the
    direct solve; symmetric pairs of D move together."""
    N, n = 6, 3
    d = lqrgen.lqr_instance(N, n, 2, 99, 0, with_target=True)
    D, O, b, t = d["D"], d["O"], d["b"], d["t"]

    def loss(D_, O_, b_):
        x_ = orc.btchol_solve(D_, O_, b_)
        return float(np.sum((x_ - t) ** 2))

    x = orc.btchol_solve(D, O, b)
    lam, dD, dO = orc.adjoint(D, O, x, 2 * (x - t))
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(12):
        which = rng.integers(3)
        if which == 0:
            k, i = rng.integers(N), rng.integers(n)
            bp, bm = b.copy(), b.copy()
            bp[k, i] += h
            bm[k, i] -= h
            fd = (loss(D, O, bp) - loss(D, O, bm)) / (2 * h)
            g = lam[k, i]
        elif which == 1:
            k, i, j = rng.integers(N), rng.integers(n), rng.integers(n)
            Dp, Dm = D.copy(), D.copy()
            for M, s in ((Dp, h), (Dm, -h)):
                M[k, i, j] += s
                if i != j:
                    M[k, j, i] += s
            fd = (loss(Dp, O, b) - loss(Dm, O, b)) / (2 * h)
            g = dD[k, i, j] + (dD[k, j, i] if i != j else 0.0)
        else:
            k, i, j = rng.integers(N - 1), rng.integers(n), rng.integers(n)
            Op, Om = O.copy(), O.copy()
            Op[k, i, j] += h
            Om[k, i, j] -= h
            fd = (loss(D, Op, b) - loss(D, Om, b)) / (2 * h)
            g = dO[k, i, j]
        assert abs(fd - g) <= max(1e-6 * abs(g), 1e-7), (which, fd, g)


# ------------------------------------------------------- initial guess x0
@pytest.mark.parametrize("kind", ["none", "opt"])
def test_pcg_from_x0_is_the_krylov_galerkin_iterate(kind):
    """PCG from x0 (textbook: r0 = b - A x0): after k steps the iterate is
    x0 + V y with V a basis of K_k(M^-1 A, M^-1 r0) and y from the Galerkin
    condition V^T (b - A (x0 + V y)) = 0, i.e. the A-norm-optimal point of
    the affine Krylov space; built densely from the paper's definitions."""
    N, n = 4, 3
    D, O = random_bt(N, n, 5)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((N, n))
    x0 = rng.standard_normal((N, n))
    A = dense_A(D, O)
    if kind == "none":
        Minv, kw = np.eye(N * n), dict(kind=orc.PC_NONE)
    else:
        G, H = G_H_ab(D, O, 1.0, -1.0)
        Minv, kw = M_inv(G, H, 2, alpha=[1.0, 7.0]), dict(m=2,
                                                          alpha=[1.0, 7.0])
    r0 = b.reshape(-1) - A @ x0.reshape(-1)
    w = Minv @ r0
    for k in (1, 2, 3, 4):
        x, info = orc.pcg(D, O, b, tol=1e-30, maxit=k, x0=x0, **kw)
        assert info["iters"] == k and info["status"] == orc.NOT_CONVERGED
        V = np.empty((N * n, k))
        v = w
        for j in range(k):
            V[:, j] = v / np.linalg.norm(v)
            v = Minv @ (A @ V[:, j])
        y = np.linalg.solve(V.T @ A @ V, V.T @ r0)
        xk = x0.reshape(-1) + V @ y
        assert np.linalg.norm(x.reshape(-1) - xk) <= \
            1e-9 * np.linalg.norm(xk), k


def test_pcg_from_x0_limits():
    D, O, b = lqr(16, 4, 2)
    A = dense_A(D, O)
    xd = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    # the solution itself: the test passes before any iteration
    x, info = orc.pcg(D, O, b, tol=1e-10, x0=xd)
    assert info["status"] == orc.OK and info["iters"] == 0
    assert np.array_equal(x, xd)
    # x0 = 0 is the default start, bit for bit
    x1, i1 = orc.pcg(D, O, b, tol=1e-10)
    x2, i2 = orc.pcg(D, O, b, tol=1e-10, x0=np.zeros_like(b))
    assert i1 == i2 and np.array_equal(x1, x2)
    # a start near the solution needs fewer iterations; the test stays
    # relative to ||b||
    rng = np.random.default_rng(4)
    xn = xd + 1e-6 * rng.standard_normal(xd.shape)
    x3, i3 = orc.pcg(D, O, b, tol=1e-10, x0=xn)
    assert i3["status"] == orc.OK and i3["iters"] < i1["iters"]
    r = np.linalg.norm(b.reshape(-1) - A @ x3.reshape(-1))
    assert r <= 1.01e-10 * np.linalg.norm(b)
