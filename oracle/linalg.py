"""Linear solves of the block-tridiagonal step system.  Test infrastructure only.

dense_solve is the plain definition x = M^{-1} rhs on the assembled
(N S) x (N S) matrix.  btd_factor / btd_solve are the block Thomas
algorithm on the same system, with partial pivoting inside each block
(LAPACK getrf: the first entry of largest magnitude wins ties) and no
pivoting across blocks.
"""

import numpy as np
import scipy.linalg


def assemble(B, a, c):
    """The full (N S) x (N S) matrix, layer-major ordering (row k*S + y)."""
    N, S, _ = B.shape
    M = np.zeros((N * S, N * S))
    for k in range(N):
        rows = slice(k * S, (k + 1) * S)
        M[rows, rows] = B[k]
        if k >= 1:
            M[rows, (k - 1) * S:k * S] = np.diag(a[k])
        if k <= N - 2:
            M[rows, (k + 1) * S:(k + 2) * S] = np.diag(c[k])
    return M


def dense_solve(B, a, c, rhs):
    N, S = rhs.shape
    return np.linalg.solve(assemble(B, a, c), rhs.reshape(N * S)).reshape(N, S)


def btd_factor(B, a, c):
    """Block Thomas elimination.

    D'_0 = B_0,  D'_k = B_k - diag(a_k) D'_{k-1}^{-1} diag(c_{k-1}),
    each D'_k factored as P L U with partial pivoting.  Returns the list of
    (lu, piv) pairs (scipy.linalg.lu_factor format)."""
    N, S, _ = B.shape
    fac = []
    for k in range(N):
        D = B[k].copy()
        if k >= 1:
            Y = scipy.linalg.lu_solve(fac[k - 1], np.diag(c[k - 1]))
            D -= a[k][:, None] * Y
        fac.append(scipy.linalg.lu_factor(D, check_finite=True))
    return fac


def btd_solve(fac, a, c, rhs):
    """Forward: g'_0 = rhs_0, g'_k = rhs_k - a_k * D'_{k-1}^{-1} g'_{k-1};
    backward: x_{N-1} = D'^{-1} g'_{N-1}, x_k = D'_k^{-1}(g'_k - c_k * x_{k+1})."""
    N, S = rhs.shape
    g = rhs.copy()
    for k in range(1, N):
        g[k] = rhs[k] - a[k] * scipy.linalg.lu_solve(fac[k - 1], g[k - 1])
    x = np.zeros_like(rhs)
    x[N - 1] = scipy.linalg.lu_solve(fac[N - 1], g[N - 1])
    for k in range(N - 2, -1, -1):
        x[k] = scipy.linalg.lu_solve(fac[k], g[k] - c[k] * x[k + 1])
    return x


def btd(B, a, c, rhs):
    return btd_solve(btd_factor(B, a, c), a, c, rhs)

