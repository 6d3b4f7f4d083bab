"""Shared test helpers: hand-built networks and small columns (inputs only)."""

import numpy as np

from synth.column import Column, make_column
from synth.network import make_network, small_network

KB_TEST = 1.380649e-16


def nasa_from_g(a6_list, a1_list=None, a7_list=None):
    """Single-range NASA-7 sets with only a1, a6, a7 (G/RT = a1(1-lnT)+a6/T-a7)."""
    S = len(a6_list)
    a1_list = a1_list or [0.0] * S
    a7_list = a7_list or [0.0] * S
    out = np.zeros((S, 2, 7))
    for y in range(S):
        for r in range(2):
            out[y, r, 0] = a1_list[y]
            out[y, r, 5] = a6_list[y]
            out[y, r, 6] = a7_list[y]
    return out


def simple_column(N, S, T=1500.0, P_top=1e-2, P_bot=1e1, Kzz=0.0, D=None,
                  alphaT=None, n0=None, mbar=2.3, g=2000.0, sigma_tau=1e-22,
                  T_profile=None):
    P = np.logspace(np.log10(P_bot), np.log10(P_top), N)
    Tk = np.full(N, T) if T_profile is None else np.asarray(T_profile, float)
    K = np.full(N, Kzz) if np.isscalar(Kzz) else np.asarray(Kzz, float)
    if n0 is None:
        n0 = np.ones((N, S))
    return Column(P_bar=P, T_K=Tk, Kzz=K, Dmol=D, alphaT=alphaT,
                  n0=np.asarray(n0, float), mbar_amu=mbar, g_cgs=g,
                  sigma_tau=sigma_tau)


def ab_network(lnA=np.log(2e-3), a6=(0.0, -500.0)):
    """A <=> B (unimolecular two-body slot with one reactant), thermo with
    G/RT = a6/T only, so k_r = k_f exp(g_B - g_A)."""
    comp = [[1, 0], [1, 0]]  # isomers: same composition
    return small_network(
        comp, ["X", "He"],
        [dict(type="bi", reac=[0], prod=[1], params=[lnA, 0.0, 0.0])],
        nasa_from_g(list(a6)), mass_amu=[10.0, 10.0])


def balanced_c1_network(max_seed=400):
    """First 12-species network with two- and three-body reactions (seed
    search from 7000) whose reactions span every non-elemental direction:
    rank(nu) = S - rank(A), so the kinetic steady state of a closed layer is
    the element-potential equilibrium.  (Two-body-only networks also conserve
    the molecule count, an extra invariant.)"""
    from oracle.rates import stoichiometry  # tests may use the oracle
    for s in range(7000, 7000 + max_seed):
        net = make_network("t12", seed=s)
        nu, _ = stoichiometry(net)
        A = net.elem_comp.astype(float)
        if np.linalg.matrix_rank(nu) == net.S - np.linalg.matrix_rank(A):
            return net
    raise RuntimeError("no full-rank network found")
