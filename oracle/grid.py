"""Column grid: densities, half levels, heights, transport coefficients, optical
depth.  Test infrastructure only.

Layer k = 0 is the bottom; k-1 and k+1 are the layers below and above, and
"k+1/2" quantities are arithmetic means of layers k and k+1 (Section 2.1,
text after Eq. discrete_continuity).
"""

from dataclasses import dataclass

import numpy as np

from .constants import KB, AMU, P_STD


@dataclass
class Grid:
    N: int
    S: int
    T: np.ndarray       # [N] K
    ngas: np.ndarray    # [N] cm^-3, n_gas = P / (k_B T)
    z: np.ndarray       # [N] cm, z_0 = 0
    dzh: np.ndarray     # [N-1] cm, z_{k+1} - z_k
    dz: np.ndarray      # [N] cm, layer thickness
    Th: np.ndarray      # [N-1] K, half-level temperature
    nh: np.ndarray      # [N-1] cm^-3, half-level n_gas
    Kh: np.ndarray      # [N-1] cm^2/s, half-level eddy coefficient
    Dh: np.ndarray      # [N-1, S] cm^2/s, half-level molecular diffusion
    beta: np.ndarray    # [N-1, S] 1/cm, drift coefficient
    tau: np.ndarray     # [N] optical depth at layer midpoints
    mix_time: float     # max over half levels/species of dzh^2 / (K + D)
    v_top: np.ndarray = None     # [S] cm/s upward escape velocity at the top
    v_dep: np.ndarray = None     # [S] cm/s deposition velocity at the bottom
    phi_surf: np.ndarray = None  # [S] cm^-2 s^-1 surface emission into the bottom layer


def make_grid(col, mass_amu):
    """Build the grid of one column.

    * n_gas,k = P_k / (k_B T_k).
    * Heights from hydrostatic balance with the mean molecular mass:
      z_{k+1} = z_k + k_B T_{k+1/2} / (mbar g) * ln(P_k / P_{k+1}).
    * dz_k = (dzh_{k-1} + dzh_k) / 2, the missing outer interval copied from
      the inner one (a single layer gets one pressure scale height).
    * beta_{y,k+1/2} = (m_y - mbar) g / (k_B T_{k+1/2})
                       + alpha_T,y (T_{k+1} - T_k) / (T_{k+1/2} dzh_k):
      the molecular-diffusion drift of Eq. transportflux written for mixing
      ratios, since 1/H_y - 1/H_o = (m_y - mbar) g / (k_B T) (Eq. dzz).
    * tau_k = sigma_tau * (n_gas,k dz_k / 2 + sum_{j>k} n_gas,j dz_j): total-gas
      column above the layer midpoint (Section 2.3.3 optical depth with a
      single gray cross section).
    """
    P = np.asarray(col.P_bar, float) * P_STD
    T = np.asarray(col.T_K, float)
    K = np.asarray(col.Kzz, float)
    N = P.shape[0]
    m = np.asarray(mass_amu, float)
    S = m.shape[0]
    D = np.zeros((N, S)) if col.Dmol is None else np.asarray(col.Dmol, float)
    alpha = np.zeros(S) if col.alphaT is None else np.asarray(col.alphaT, float)
    mbar = col.mbar_amu * AMU
    g = col.g_cgs

    ngas = P / (KB * T)
    Th = 0.5 * (T[:-1] + T[1:])
    nh = 0.5 * (ngas[:-1] + ngas[1:])
    Kh = 0.5 * (K[:-1] + K[1:])
    Dh = 0.5 * (D[:-1] + D[1:])

    z = np.zeros(N)
    for k in range(N - 1):
        z[k + 1] = z[k] + KB * Th[k] / (mbar * g) * np.log(P[k] / P[k + 1])
    dzh = z[1:] - z[:-1]

    dz = np.zeros(N)
    if N == 1:
        # A single layer has no neighbours; its thickness is taken as one
        # pressure scale height k_B T / (mbar g) (only tau uses it).
        dz[0] = KB * T[0] / (mbar * g)
    for k in range(N if N > 1 else 0):
        below = dzh[k - 1] if k >= 1 else dzh[k]
        above = dzh[k] if k <= N - 2 else dzh[k - 1]
        dz[k] = 0.5 * (below + above)

    beta = np.zeros((N - 1, S))
    for k in range(N - 1):
        beta[k] = ((m * AMU - mbar) * g / (KB * Th[k])
                   + alpha * (T[k + 1] - T[k]) / (Th[k] * dzh[k]))

    tau = np.zeros(N)
    for k in range(N):
        col_above = 0.5 * ngas[k] * dz[k] + sum(ngas[j] * dz[j] for j in range(k + 1, N))
        tau[k] = col.sigma_tau * col_above

    mix = 0.0
    for k in range(N - 1):
        for y in range(S):
            kd = Kh[k] + Dh[k, y]
            if kd > 0.0:
                mix = max(mix, dzh[k] ** 2 / kd)

    v_top, v_dep, phi_surf = boundary_velocities(col, T, D, m, mbar, g)
    return Grid(N=N, S=S, T=T, ngas=ngas, z=z, dzh=dzh, dz=dz, Th=Th, nh=nh,
                Kh=Kh, Dh=Dh, beta=beta, tau=tau, mix_time=mix, v_top=v_top,
                v_dep=v_dep, phi_surf=phi_surf)


def boundary_velocities(col, T, D, m_amu, mbar, g):
    """Boundary exchange of the column (zero everywhere when closed).

    Top (Section 2.4): species flagged in col.escape_diff_limited leave with
    the diffusion-limited velocity V_lim = D (1/H_0 - 1/H_y), H_0 = k_B T /
    (mbar g) the atmosphere's and H_y = k_B T / (m_y g) the species' scale
    height.  Readings: D and T are the top layer's (no half level lies above
    it), and V_lim < 0 (a species heavier than the mean) gives no escape.
    col.v_top adds set velocities (the paper's user-defined escape).
    Bottom (Section 2.5): deposition velocities col.v_dep and surface
    emission fluxes col.phi_surf."""
    S = m_amu.shape[0]
    v_top = np.zeros(S)
    flags = getattr(col, "escape_diff_limited", None)
    if flags is not None:
        H0 = KB * T[-1] / (mbar * g)
        for y in range(S):
            if flags[y]:
                Hy = KB * T[-1] / (m_amu[y] * AMU * g)
                v_top[y] = max(D[-1, y] * (1.0 / H0 - 1.0 / Hy), 0.0)
    extra = getattr(col, "v_top", None)
    if extra is not None:
        v_top = v_top + np.asarray(extra, float)
    v_dep = getattr(col, "v_dep", None)
    v_dep = np.zeros(S) if v_dep is None else np.asarray(v_dep, float).copy()
    phi = getattr(col, "phi_surf", None)
    phi = np.zeros(S) if phi is None else np.asarray(phi, float).copy()
    return v_top, v_dep, phi
