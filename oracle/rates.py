"""Rate coefficients (Section 2.3).  Test infrastructure only.

params[r] layout per reaction type:
  two-body   (ln alpha, beta, gamma, -, -, -)
  three-body (ln alpha0, beta0, gamma0, ln alpha_inf, beta_inf, gamma_inf)
  photolysis (ln J0, -, -, -, -, -)
"""

import numpy as np

from .constants import KB, P_STD
from .thermo import species_g

RT_BIMOL, RT_TERMOL, RT_PHOTO = 0, 1, 2


def arrhenius(ln_alpha, beta, gamma, T, kooij):
    """Section 2.3.1: k = alpha T_b^beta exp(-gamma / T), T_b = T/300 for the
    Kooij form and T_b = T for the modified Arrhenius form."""
    Tb = np.where(kooij, T / 300.0, T)
    return np.exp(ln_alpha) * Tb ** beta * np.exp(-gamma / T)


def lindemann(k0, kinf, M):
    """Section 2.3.2: k = k0 [M] / (1 + k0 [M] / k_inf)."""
    return k0 * M / (1.0 + k0 * M / kinf)


def photolysis(ln_J0, tau):
    """Section 2.3.3 with a gray flux: k_ph = t_f J0 exp(-tau / mu), t_f = mu = 1
    and no diffuse component."""
    return np.exp(ln_J0) * np.exp(-tau)


def forward_rates(net, grid):
    """k_f[k, r] for every layer and reaction.  The third body is the total gas,
    [M] = n_gas,k, with unit efficiency for every species."""
    N, R = grid.N, net.rtype.shape[0]
    p = np.asarray(net.params, float)
    kooij = np.asarray(net.tb_kooij, bool)
    t = np.asarray(net.rtype)
    kf = np.zeros((N, R))
    for k in range(N):
        T, M, tau = grid.T[k], grid.ngas[k], grid.tau[k]
        two = arrhenius(p[:, 0], p[:, 1], p[:, 2], T, kooij)
        k0 = two    # three-body low-pressure law sits in the same slots
        kinf = arrhenius(p[:, 3], p[:, 4], p[:, 5], T, kooij)
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            three = lindemann(k0, kinf, M)
            photo = photolysis(p[:, 0], tau)
        kf[k] = np.where(t == RT_BIMOL, two, np.where(t == RT_TERMOL, three, photo))
    return kf


def stoichiometry(net):
    """Net stoichiometric matrix nu[r, y] = (times y is a product) - (times y is
    a reactant), and Delta nu[r] = #products - #reactants (the third body M
    is never listed)."""
    R, S = net.rtype.shape[0], net.nasa7.shape[0]
    nu = np.zeros((R, S))
    dnu = np.zeros(R)
    for r in range(R):
        for y in net.prod[r]:
            if y >= 0:
                nu[r, y] += 1.0
                dnu[r] += 1.0
        for y in net.reac[r]:
            if y >= 0:
                nu[r, y] -= 1.0
                dnu[r] -= 1.0
    return nu, dnu


def reverse_rates(net, grid, kf):
    """Section 2.3.4: k_r = k_f / K_c with the equilibrium constant from the
    reaction Gibbs energy, K_c = exp(-Delta g) (P0 / (k_B T))^Delta nu,
    Delta g = sum_products G/RT - sum_reactants G/RT (concentrations in
    cm^-3, standard state 1 bar).  Photolysis and any reaction flagged
    irreversible get k_r = 0."""
    N, R = kf.shape
    nu, dnu = stoichiometry(net)
    rev = (np.asarray(net.reversible) != 0) & (np.asarray(net.rtype) != RT_PHOTO)
    kr = np.zeros((N, R))
    for k in range(N):
        T = grid.T[k]
        dg = nu @ species_g(net.nasa7, net.t_mid, T)
        Kc = np.exp(-dg) * (P_STD / (KB * T)) ** dnu
        kr[k] = np.where(rev, kf[k] / Kc, 0.0)
    return kr


def rates(net, grid):
    kf = forward_rates(net, grid)
    return kf, reverse_rates(net, grid, kf)
