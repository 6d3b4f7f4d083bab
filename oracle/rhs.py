"""Right-hand side of the continuity equation.  Test infrastructure only.

Eq. continuity: dn_y/dt = P_y - L_y - d(phi_y)/dz.
"""

import numpy as np


def reaction_rates(net, kf, kr, n):
    """w[k, r] = k_f prod_{reactants} n - k_r prod_{products} n; a species
    listed twice enters squared (e.g. 2 SO)."""
    N, R = kf.shape
    fwd = np.ones((N, R))
    rev = np.ones((N, R))
    for j in range(net.reac.shape[1]):
        idx = net.reac[:, j]
        on = idx >= 0
        fwd[:, on] *= n[:, idx[on]]
    for j in range(net.prod.shape[1]):
        idx = net.prod[:, j]
        on = idx >= 0
        rev[:, on] *= n[:, idx[on]]
    return kf * fwd - kr * rev


def chem_rhs(net, w, S):
    """f_chem[k, y] = sum_r (nu+_{y,r} - nu-_{y,r}) w[k, r] (production minus
    loss, Eq. continuity)."""
    N, R = w.shape
    f = np.zeros((N, S))
    for r in range(R):
        for y in net.prod[r]:
            if y >= 0:
                f[:, y] += w[:, r]
        for y in net.reac[r]:
            if y >= 0:
                f[:, y] -= w[:, r]
    return f


def half_level_flux(grid, n):
    """Upward-positive mixing-ratio flux F = -phi at the N-1 interior half
    levels, from Eq. transportflux with y = n / n_gas:

      phi_y = -n_gas [ (K + D) dy/dz + D beta_y y ],
      F_{k+1/2} = n_gas,k+1/2 [ (K + D)_{k+1/2} (y_{k+1} - y_k) / dzh_k
                                + D_{k+1/2} beta_{k+1/2} (y_k + y_{k+1}) / 2 ].

    The eddy term of Eq. transportflux equals -K n_gas dy/dz exactly for a
    hydrostatic ideal gas, since d ln n_gas / dz = -1/H_o - T'/T."""
    y = n / grid.ngas[:, None]
    F = np.zeros((grid.N - 1, n.shape[1]))
    for k in range(grid.N - 1):
        KD = grid.Kh[k] + grid.Dh[k]
        F[k] = grid.nh[k] * (KD * (y[k + 1] - y[k]) / grid.dzh[k]
                             + grid.Dh[k] * grid.beta[k] * 0.5 * (y[k] + y[k + 1]))
    return F


def boundary_flux(grid, n):
    """F (= -phi, upward-positive phi) through the bottom and top of the
    column: phi_bottom = phi_surf - v_dep n_0 (emission up, deposition down),
    phi_top = v_top n_{N-1} (escape up); zero for a closed column
    (Sections 2.4, 2.5)."""
    zero = np.zeros(n.shape[1])
    v_top = zero if grid.v_top is None else grid.v_top
    v_dep = zero if grid.v_dep is None else grid.v_dep
    phi = zero if grid.phi_surf is None else grid.phi_surf
    F_bottom = -(phi - v_dep * n[0])
    F_top = -(v_top * n[grid.N - 1])
    return F_bottom, F_top


def transport_rhs(grid, n):
    """-d(phi)/dz at layer k = (F_{k+1/2} - F_{k-1/2}) / dz_k, the outermost
    F being the boundary fluxes."""
    F = half_level_flux(grid, n)
    F_bottom, F_top = boundary_flux(grid, n)
    f = np.zeros_like(n)
    for k in range(grid.N):
        up = F[k] if k <= grid.N - 2 else F_top
        down = F[k - 1] if k >= 1 else F_bottom
        f[k] = (up - down) / grid.dz[k]
    return f


def rhs(net, grid, kf, kr, n):
    w = reaction_rates(net, kf, kr, n)
    return chem_rhs(net, w, n.shape[1]) + transport_rhs(grid, n)
