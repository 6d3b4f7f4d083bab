"""Pins for the oracle's grid and transport (CPU only)."""

import numpy as np
import pytest
import scipy.linalg

from oracle import grid as grid_mod, rhs as rhs_mod, jacobian, linalg
from oracle.constants import KB, AMU
from tests.helpers import simple_column


def test_isothermal_heights_are_scale_height_logs():
    col = simple_column(30, 2, T=1200.0, P_bot=100.0, P_top=1e-6)
    g = grid_mod.make_grid(col, np.array([2.0, 30.0]))
    H = KB * 1200.0 / (col.mbar_amu * AMU * col.g_cgs)
    P = col.P_bar
    np.testing.assert_allclose(g.z, H * np.log(P[0] / P), rtol=1e-12, atol=1e-6)


def test_layer_thickness_rule():
    col = simple_column(7, 1, T_profile=np.linspace(2000, 1000, 7))
    g = grid_mod.make_grid(col, np.array([2.0]))
    np.testing.assert_allclose(g.dz[1:-1], 0.5 * (g.dzh[:-1] + g.dzh[1:]), rtol=1e-15)
    assert g.dz[0] == g.dzh[0] and g.dz[-1] == g.dzh[-1]


def test_optical_depth_matches_hydrostatic_column():
    # In hydrostatic balance the gas column above level k is P_k / (mbar g);
    # the discrete sum approximates it to grid accuracy on a fine grid.
    N = 400
    col = simple_column(N, 1, T_profile=np.linspace(2000, 1000, N), P_bot=100.0, P_top=1e-8)
    g = grid_mod.make_grid(col, np.array([2.0]))
    hydro = col.P_bar * 1e6 / (col.mbar_amu * AMU * col.g_cgs) * col.sigma_tau
    deep = col.P_bar > 1e3 * col.P_bar[-1]
    np.testing.assert_allclose(g.tau[deep], hydro[deep], rtol=0.02)


def _diffusive_column(N=12, S=3, alpha=True):
    T = np.linspace(1800, 900, N)
    P = np.logspace(1, -5, N)
    masses = np.array([2.0, 18.0, 44.0])[:S]
    D = 1e21 * (T[:, None] / 1000) ** 0.7 * np.sqrt(2.0 / masses)[None, :] / (P[:, None] * 1e6 / (KB * T[:, None]))
    col = simple_column(N, S, T_profile=T, P_bot=10.0, P_top=1e-5,
                        Kzz=np.logspace(7, 9, N), D=D,
                        alphaT=np.array([-0.38, 0.1, 0.3])[:S] if alpha else None)
    return col, masses


def test_zero_flux_boundaries_conserve_column():
    # sum_k dz_k f_tr,k telescopes to F_{N-1/2} - F_{-1/2} = 0.
    col, m = _diffusive_column()
    g = grid_mod.make_grid(col, m)
    rng = np.random.default_rng(3)
    n = g.ngas[:, None] * 10.0 ** rng.uniform(-12, -1, (g.N, 3))
    f = rhs_mod.transport_rhs(g, n)
    total = np.abs(g.dz[:, None] * f).sum(axis=0)
    assert np.all(np.abs((g.dz[:, None] * f).sum(axis=0)) <= 1e-13 * total)


def test_eddy_only_uniform_mixing_ratio_is_stationary():
    col = simple_column(15, 2, T_profile=np.linspace(2000, 1000, 15), Kzz=np.logspace(7, 10, 15))
    g = grid_mod.make_grid(col, np.array([2.0, 30.0]))
    n = g.ngas[:, None] * np.array([[0.3, 1e-7]])
    f = rhs_mod.transport_rhs(g, n)
    scale = (g.Kh[0] * g.ngas[0] / g.dzh[0] ** 2)
    assert np.max(np.abs(f)) <= 1e-13 * scale


def test_discrete_diffusive_equilibrium_has_zero_flux():
    # With D > 0 the flux vanishes where
    # y_{k+1}/y_k = ((K+D)/dzh - D beta/2) / ((K+D)/dzh + D beta/2).
    col, m = _diffusive_column()
    g = grid_mod.make_grid(col, m)
    y = np.ones((g.N, 3))
    for k in range(g.N - 1):
        KD = g.Kh[k] + g.Dh[k]
        y[k + 1] = y[k] * (KD / g.dzh[k] - 0.5 * g.Dh[k] * g.beta[k]) / (KD / g.dzh[k] + 0.5 * g.Dh[k] * g.beta[k])
    n = y * g.ngas[:, None] * 1e-6
    F = rhs_mod.half_level_flux(g, n)
    # scale of the individual terms (the flux is their cancellation)
    parts = g.nh[:, None] * (g.Kh[:, None] + g.Dh) * (y[1:] + y[:-1]) * 1e-6 / g.dzh[:, None]
    assert np.all(np.abs(F) <= 1e-13 * parts)
    assert np.all(np.abs(rhs_mod.transport_rhs(g, n)[:-1]) <= 1e-12 * parts / g.dz[:-1, None])


def test_transport_jacobian_is_exact_linearisation():
    col, m = _diffusive_column()
    g = grid_mod.make_grid(col, m)
    lower, diag, upper = jacobian.transport_coefficients(g)
    rng = np.random.default_rng(5)
    n = g.ngas[:, None] * 10.0 ** rng.uniform(-8, -1, (g.N, 3))
    f = rhs_mod.transport_rhs(g, n)
    pred = diag * n
    pred[1:] += lower[1:] * n[:-1]
    pred[:-1] += upper[:-1] * n[1:]
    np.testing.assert_allclose(pred, f, rtol=1e-9, atol=1e-12 * np.abs(f).max())


def test_single_species_diffusion_step_equals_banded_solve():
    # A BE step for one inert species with transport only is a tridiagonal
    # solve; scipy.linalg.solve_banded must give the same increment.
    col, m = _diffusive_column(S=1)
    g = grid_mod.make_grid(col, m)
    lower, diag, upper = jacobian.transport_coefficients(g)
    n = g.ngas[:, None] * np.linspace(1e-3, 1e-6, g.N)[:, None]
    dt = 3.0e5
    f = rhs_mod.transport_rhs(g, n)
    B = np.zeros((g.N, 1, 1))
    B[:, 0, 0] = 1.0 / dt - diag[:, 0]
    x = linalg.btd(B, -lower, -upper, f)
    ab = np.zeros((3, g.N))
    ab[0, 1:] = -upper[:-1, 0]
    ab[1, :] = 1.0 / dt - diag[:, 0]
    ab[2, :-1] = -lower[1:, 0]
    ref = scipy.linalg.solve_banded((1, 1), ab, f[:, 0])
    np.testing.assert_allclose(x[:, 0], ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_eddy_only_relaxes_to_uniform_mixing_ratio():
    # Without chemistry and molecular diffusion the steady state has a uniform
    # mixing ratio y = sum n dz / sum n_gas dz (column conservation).
    col = simple_column(10, 1, T_profile=np.linspace(2000, 1000, 10), Kzz=1e8, P_bot=1.0, P_top=1e-3)
    g = grid_mod.make_grid(col, np.array([16.0]))
    n = g.ngas[:, None] * np.linspace(1e-3, 1e-9, 10)[:, None]
    expect = (n[:, 0] * g.dz).sum() / (g.ngas * g.dz).sum()
    lower, diag, upper = jacobian.transport_coefficients(g)
    for dt in [1e4 * 2 ** j for j in range(40)]:
        B = np.zeros((10, 1, 1))
        B[:, 0, 0] = 1.0 / dt - diag[:, 0]
        n = n + linalg.btd(B, -lower, -upper, rhs_mod.transport_rhs(g, n))
    np.testing.assert_allclose(n[:, 0] / g.ngas, expect, rtol=1e-9)
