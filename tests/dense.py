"""Dense matrices built directly from the paper's definitions (test side).

Independent of the C oracle: these are assembled entry by entry from eq. (1)
and the splitting pictures of Section II-C, then handled with numpy's dense
linear algebra. Tests use them to pin the oracle.
"""
import numpy as np


def dense_A(D, O):
    """Eq. (1): D_k on the diagonal, O_k at (k,k+1), O_k^T at (k+1,k)."""
    N, n = D.shape[0], D.shape[1]
    A = np.zeros((N * n, N * n))
    for k in range(N):
        A[k * n:(k + 1) * n, k * n:(k + 1) * n] = D[k]
    for k in range(N - 1):
        A[k * n:(k + 1) * n, (k + 1) * n:(k + 2) * n] = O[k]
        A[(k + 1) * n:(k + 2) * n, k * n:(k + 1) * n] = O[k].T
    return A


def _blk(M, n, i, j):
    return M[i * n:(i + 1) * n, j * n:(j + 1) * n]


def splittings(D, O):
    """B_d, C_d (eq. def-diagonal-splitting) and B_l, C_l, B_r, C_r
    (eq. def-stair-splittings), each drawn from the paper's pictures.

    With 1-based block rows as in the paper: B_l keeps the full rows 2, 4, ...
    and C_l holds -O blocks in rows 1, 3, ...; B_r keeps the full rows
    1, 3, ... and C_r holds -O blocks in rows 2, 4, ....
    """
    N, n = D.shape[0], D.shape[1]
    size = N * n
    S = {key: np.zeros((size, size)) for key in
         ("Bd", "Cd", "Bl", "Cl", "Br", "Cr")}
    for k in range(N):                       # 0-based k is paper row k+1
        paper_even = (k + 1) % 2 == 0
        for key in ("Bd", "Bl", "Br"):
            _blk(S[key], n, k, k)[:] = D[k]
        left = k - 1 >= 0
        right = k + 1 <= N - 1
        # off-diagonal entries of block row k of A
        offs = []
        if left:
            offs.append((k - 1, O[k - 1].T))
        if right:
            offs.append((k + 1, O[k]))
        for j, blk in offs:
            _blk(S["Cd"], n, k, j)[:] = -blk
            if paper_even:
                _blk(S["Bl"], n, k, j)[:] = blk
                _blk(S["Cr"], n, k, j)[:] = -blk
            else:
                _blk(S["Br"], n, k, j)[:] = blk
                _blk(S["Cl"], n, k, j)[:] = -blk
    return S


def G_H_ab(D, O, a, b):
    """Eq. (def-GH-ab-multi-splitting) with dense inverses."""
    S = splittings(D, O)
    iBl, iBr, iBd = (np.linalg.inv(S[k]) for k in ("Bl", "Br", "Bd"))
    G = a * (iBl + iBr) + b * iBd
    H = a * (iBl @ S["Cl"] + iBr @ S["Cr"]) + b * iBd @ S["Cd"]
    return G, H


def M_inv(G, H, m, alpha=None):
    """Eqs. (Mabinv) / (Mminv-polynomial-coefficients), dense."""
    size = G.shape[0]
    P = np.eye(size)
    Hp = np.eye(size)
    for i in range(1, m):
        Hp = Hp @ H
        c = 1.0 if alpha is None else float(alpha[i])
        P = P + c * Hp
    return P @ G


def random_bt(N, n, seed, off=0.6):
    """Generic random SPD block-tridiagonal matrix (not LQR-shaped)."""
    rng = np.random.default_rng(seed)
    D = np.empty((N, n, n))
    for k in range(N):
        M = rng.standard_normal((n, n))
        D[k] = M @ M.T / n + np.eye(n)
    O = off * rng.standard_normal((max(N - 1, 0), n, n)) / np.sqrt(n)
    for _ in range(60):
        if N == 1 or np.linalg.eigvalsh(dense_A(D, O)).min() > 1e-3:
            break
        O *= 0.7
    return D, O


def blocks_of(Mat, N, n):
    """(N, n) view helpers: vector <-> block vector."""
    return Mat.reshape(N, n)


def op_matrix(apply, N, n):
    """Dense matrix of a linear map given as apply(v (N,n)) -> (N,n)."""
    size = N * n
    M = np.empty((size, size))
    for j in range(size):
        e = np.zeros(size)
        e[j] = 1.0
        M[:, j] = apply(e.reshape(N, n)).reshape(-1)
    return M
