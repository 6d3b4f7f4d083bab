"""Pins for the oracle's thermochemistry and rate laws (CPU only)."""

import os

import numpy as np
import pytest

from oracle import thermo, rates, grid as grid_mod
from oracle.constants import KB, P_STD
from tests.helpers import simple_column, nasa_from_g
from synth.network import small_network

GOLD = os.path.join(os.path.dirname(__file__), "golden", "nasa7_table.txt")
R_GAS = 8.314462618  # J/(mol K), exact SI value


def table():
    out = {}
    for line in open(GOLD):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        out.setdefault(f[0], {})[f[1]] = np.array([float(x) for x in f[2:]])
    return out


@pytest.mark.parametrize("mol", ["H2O_burcat", "CO2_burcat", "H2O_thiswork", "P2D"])
def test_g_over_rt_continuous_at_tmid(mol):
    # Appendix A table: the low (to 1000 K) and high (from 1000 K) fits of the
    # same molecule must give the same G/RT at 1000 K.  A wrong sign or divisor
    # in any term of the polynomial breaks this (the two sets differ).
    t = table()[mol]
    lo = thermo.g_over_rt(t["low"], 1000.0)
    hi = thermo.g_over_rt(t["high"], 1000.0)
    assert abs(lo - hi) <= 5e-6 * abs(lo)


@pytest.mark.parametrize("mol", ["H2O_burcat", "CO2_burcat", "P2D"])
def test_cp_over_r_continuous_at_tmid(mol):
    t = table()[mol]
    lo = thermo.cp_over_r(t["low"], 1000.0)
    hi = thermo.cp_over_r(t["high"], 1000.0)
    assert abs(lo - hi) <= 5e-5 * abs(lo)


@pytest.mark.parametrize("mol,dfh_kj,s_j,cp_j", [
    # CODATA key values for thermodynamics (gas, 298.15 K, 1 bar):
    # H2O: dfH = -241.826 kJ/mol, S = 188.835 J/(mol K), Cp = 33.58 J/(mol K)
    # CO2: dfH = -393.51 kJ/mol,  S = 213.785 J/(mol K), Cp = 37.12 J/(mol K)
    ("H2O_burcat", -241.826, 188.835, 33.58),
    ("CO2_burcat", -393.51, 213.785, 37.12),
])
def test_g_over_rt_reproduces_codata_at_298(mol, dfh_kj, s_j, cp_j):
    a = table()[mol]["low"]
    T = 298.15
    expect = dfh_kj * 1e3 / (R_GAS * T) - s_j / R_GAS
    assert thermo.g_over_rt(a, T) == pytest.approx(expect, rel=2e-5)
    assert thermo.cp_over_r(a, T) * R_GAS == pytest.approx(cp_j, rel=2e-3)


def test_species_g_range_switch_at_tmid():
    t = table()["H2O_burcat"]
    nasa = np.stack([np.stack([t["low"], t["high"]])])
    assert thermo.species_g(nasa, 1000.0, 999.0)[0] == thermo.g_over_rt(t["low"], 999.0)
    assert thermo.species_g(nasa, 1000.0, 1000.0)[0] == thermo.g_over_rt(t["high"], 1000.0)


def test_arrhenius_closed_forms():
    A = 3.0e-12
    for kooij in (False, True):
        assert rates.arrhenius(np.log(A), 0.0, 0.0, 1234.0, kooij) == pytest.approx(A, rel=1e-14)
    # Kooij at T = 300 K: T_b = 1 so the beta term vanishes.
    assert rates.arrhenius(np.log(A), 1.7, 900.0, 300.0, True) == pytest.approx(
        A * np.exp(-3.0), rel=1e-14)
    # Modified Arrhenius with beta = 1, gamma = 0: k = A T.
    assert rates.arrhenius(np.log(A), 1.0, 0.0, 1500.0, False) == pytest.approx(A * 1500.0, rel=1e-14)
    # Kooij with beta = 2: k = A (T/300)^2.
    assert rates.arrhenius(np.log(A), 2.0, 0.0, 1500.0, True) == pytest.approx(A * 25.0, rel=1e-14)


def test_lindemann_limits():
    k0, kinf = 1e-30, 1e-11
    assert rates.lindemann(k0, kinf, 1e3) == pytest.approx(k0 * 1e3, rel=1e-12)
    assert rates.lindemann(k0, kinf, 1e40) == pytest.approx(kinf, rel=1e-9)
    assert rates.lindemann(k0, kinf, kinf / k0) == pytest.approx(kinf / 2.0, rel=1e-14)


def test_photolysis_gray():
    assert rates.photolysis(np.log(1e-4), 0.0) == pytest.approx(1e-4, rel=1e-14)
    assert rates.photolysis(np.log(1e-4), 2.0) == pytest.approx(1e-4 * np.exp(-2.0), rel=1e-14)


def _hand_net():
    # species: 0 A, 1 B, 2 C(=A+B), 3 D; compositions over (X, Y)
    comp = [[1, 0], [0, 1], [1, 1], [0, 1]]
    rx = [
        dict(type="bi", reac=[0, 1], prod=[2], params=[np.log(2e-11), 0.5, 800.0]),
        dict(type="ter", reac=[0, 1], prod=[2],
             params=[np.log(3e-30), -1.0, 100.0, np.log(4e-11), 0.2, 50.0], kooij=True),
        dict(type="ph", reac=[2], prod=[0, 1], params=[np.log(5e-5)]),
    ]
    return small_network(comp, ["X", "Y"], rx,
                         nasa_from_g([1000.0, -2000.0, -9000.0, 0.0]),
                         mass_amu=[10.0, 12.0, 22.0, 12.0])


def test_forward_rates_by_type_and_layer():
    net = _hand_net()
    col = simple_column(5, 4, T_profile=[1800, 1600, 1400, 1200, 1000], P_bot=10.0, P_top=1e-3)
    g = grid_mod.make_grid(col, net.mass_amu)
    kf = rates.forward_rates(net, g)
    for k in range(5):
        T, M = g.T[k], g.ngas[k]
        assert kf[k, 0] == pytest.approx(2e-11 * T ** 0.5 * np.exp(-800.0 / T), rel=1e-13)
        k0 = 3e-30 * (T / 300.0) ** -1.0 * np.exp(-100.0 / T)
        ki = 4e-11 * (T / 300.0) ** 0.2 * np.exp(-50.0 / T)
        assert kf[k, 1] == pytest.approx(k0 * M / (1.0 + k0 * M / ki), rel=1e-13)
        assert kf[k, 2] == pytest.approx(5e-5 * np.exp(-g.tau[k]), rel=1e-13)


def test_reverse_rates_from_gibbs():
    net = _hand_net()
    col = simple_column(3, 4, T_profile=[1500, 1000, 900])
    g = grid_mod.make_grid(col, net.mass_amu)
    kf, kr = rates.rates(net, g)
    for k in range(3):
        T = g.T[k]
        gy = np.array([1000.0, -2000.0, -9000.0, 0.0]) / T
        # A + B -> C: Delta nu = -1, K_c = exp(-(gC - gA - gB)) * kB T / P0
        Kc = np.exp(-(gy[2] - gy[0] - gy[1])) * (KB * T / P_STD)
        assert kf[k, 0] / kr[k, 0] == pytest.approx(Kc, rel=1e-12)
        assert kf[k, 1] / kr[k, 1] == pytest.approx(Kc, rel=1e-12)
        assert kr[k, 2] == 0.0   # photolysis is irreversible
