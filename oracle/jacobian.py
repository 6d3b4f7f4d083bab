"""Jacobian of the right-hand side and the block-tridiagonal step matrix.
Test infrastructure only.

The step matrix of the linearly implicit backward-Euler step is
M = I/dt - dF/dn.  Ordered layer by layer it is block tridiagonal: the
chemistry couples species within a layer (dense S x S diagonal blocks) and
transport couples each species only with itself in the layers below and
above (diagonal off-diagonal blocks), cf. Eq. discrete_continuity.

Block row k reads   a_k * x_{k-1} + B_k x_k + c_k * x_{k+1} = rhs_k
with a_k, c_k vectors (diagonal blocks) and B_k dense.
"""

import numpy as np


def chem_jacobian(net, kf, kr, n):
    """J[k, y, x] = d f_chem[k, y] / d n[k, x], analytic:
    dw_r/dn_x = k_f m_x n_x^(m_x - 1) prod_{other reactants} n
              - k_r m'_x n_x^(m'_x - 1) prod_{other products} n."""
    N, S = n.shape
    R = kf.shape[0 if kf.ndim == 1 else 1]
    J = np.zeros((N, S, S))
    for r in range(R):
        reac = [y for y in net.reac[r] if y >= 0]
        prod = [y for y in net.prod[r] if y >= 0]
        nu = {}
        for y in prod:
            nu[y] = nu.get(y, 0) + 1
        for y in reac:
            nu[y] = nu.get(y, 0) - 1
        for side, kcoef, sign in ((reac, kf[:, r], 1.0), (prod, kr[:, r], -1.0)):
            for x in set(side):
                m = side.count(x)
                dprod = m * n[:, x] ** (m - 1)
                for y in side:
                    if y != x:
                        dprod = dprod * n[:, y]
                dw = sign * kcoef * dprod
                for y, v in nu.items():
                    if v != 0:
                        J[:, y, x] += v * dw
    return J


def transport_coefficients(grid):
    """Linear transport coefficients of f_tr (Eq. transportflux discretised):

      p_k = dF_{k+1/2}/dn_{k+1} = n_h [ (K+D)/dzh + D beta / 2 ] / n_gas,k+1
      q_k = dF_{k+1/2}/dn_k     = n_h [ -(K+D)/dzh + D beta / 2 ] / n_gas,k

    so that df_tr,k/dn_{k+1} = p_k / dz_k, df_tr,k/dn_{k-1} = -q_{k-1} / dz_k,
    df_tr,k/dn_k = (q_k - p_{k-1}) / dz_k; the boundary fluxes add
    -v_dep / dz_0 at the bottom and -v_top / dz_{N-1} at the top (their
    surface emission is constant).
    Returns (lower, diag, upper) arrays [N, S] of these derivatives."""
    N, S = grid.N, grid.S
    p = np.zeros((N - 1, S))
    q = np.zeros((N - 1, S))
    for k in range(N - 1):
        KD = grid.Kh[k] + grid.Dh[k]
        half = 0.5 * grid.Dh[k] * grid.beta[k]
        p[k] = grid.nh[k] * (KD / grid.dzh[k] + half) / grid.ngas[k + 1]
        q[k] = grid.nh[k] * (-KD / grid.dzh[k] + half) / grid.ngas[k]
    lower = np.zeros((N, S))
    diag = np.zeros((N, S))
    upper = np.zeros((N, S))
    for k in range(N):
        if k >= 1:
            lower[k] = -q[k - 1] / grid.dz[k]
            diag[k] -= p[k - 1] / grid.dz[k]
        if k <= N - 2:
            upper[k] = p[k] / grid.dz[k]
            diag[k] += q[k] / grid.dz[k]
    if grid.v_dep is not None:
        diag[0] -= grid.v_dep / grid.dz[0]
    if grid.v_top is not None:
        diag[N - 1] -= grid.v_top / grid.dz[N - 1]
    return lower, diag, upper


def step_matrix(net, grid, kf, kr, n, dt):
    """Blocks of M = I/dt - dF/dn: B [N, S, S], a [N, S], c [N, S]."""
    N, S = n.shape
    J = chem_jacobian(net, kf, kr, n)
    lower, diag, upper = transport_coefficients(grid)
    B = -J
    for k in range(N):
        B[k] += np.eye(S) / dt - np.diag(diag[k])
    return B, -lower, -upper
