"""Pins of the oracle's boundary exchange (Section 2.4 escape with the
diffusion-limited velocity, Section 2.5 deposition and surface emission).

* Column budget: the interior fluxes telescope, so with the chemistry off
  sum_k f[k] dz_k equals the net boundary inflow phi_surf - v_dep n_0 -
  v_top n_{N-1} of every species, for any state.
* Exact steady states of the linear transport problem (a backward-Euler
  step with dt = 1e30 from an empty column lands on them): emission
  balanced by deposition gives v_dep n_0 = phi_surf; emission carried out
  by escape gives v_top n_{N-1} = phi_surf.
* V_lim in its mass-difference form D (mbar - m_y) g / (k_B T) at the top
  layer, zero for heavier-than-mean or unflagged species.
* The step matrix's boundary rows are the derivative of the right-hand side
  (central differences of the linear transport problem)."""

import dataclasses

import numpy as np
import pytest

import synth
from oracle import grid as grid_mod
from oracle import integrate
from oracle.constants import AMU, KB


@pytest.fixture(scope="module")
def net_col():
    net, col = synth.make_config(2)
    return net, synth.with_boundary(net, col)


def transport_only(net, col):
    prob = integrate.Problem(net, col)
    prob.kf = np.zeros_like(prob.kf)
    prob.kr = np.zeros_like(prob.kr)
    return prob


def test_boundary_recipe_opens_both_ends(net_col):
    net, col = net_col
    g = grid_mod.make_grid(col, net.mass_amu)
    assert (g.v_top > 0).sum() >= 3 and (g.v_dep > 0).sum() >= 10 and (g.phi_surf > 0).sum() >= 5


def test_column_budget_is_the_boundary_inflow(net_col):
    net, col = net_col
    prob = transport_only(net, col)
    g = prob.grid
    n = col.n0 * (1.0 + 0.5 * np.random.default_rng(5).random(col.n0.shape))
    f = prob.rhs(n)
    budget = (f * g.dz[:, None]).sum(axis=0)
    inflow = g.phi_surf - g.v_dep * n[0] - g.v_top * n[-1]
    scale = (np.abs(f) * g.dz[:, None]).sum(axis=0) + np.abs(g.phi_surf) \
        + g.v_dep * n[0] + g.v_top * n[-1]
    assert np.all(np.abs(budget - inflow) <= 1e-12 * scale)
    assert np.abs(inflow).max() > 0


def test_closed_column_conserves_every_species(net_col):
    net, col = net_col
    closed = dataclasses.replace(col, escape_diff_limited=None, v_top=None, v_dep=None,
                                 phi_surf=None)
    prob = transport_only(net, closed)
    n = col.n0 * (1.0 + 0.5 * np.random.default_rng(6).random(col.n0.shape))
    f = prob.rhs(n)
    budget = (f * prob.grid.dz[:, None]).sum(axis=0)
    assert np.all(np.abs(budget) <= 1e-12 * (np.abs(f) * prob.grid.dz[:, None]).sum(axis=0))


def test_steady_state_deposits_what_the_surface_emits(net_col):
    """Emission and deposition at the bottom only: the steady column returns
    to the surface what it emits, v_dep n_0 = phi_surf (from an empty column,
    one backward-Euler step at dt = 1e30 of the linear problem)."""
    net, col = net_col
    S = len(net.mass_amu)
    v_dep = np.full(S, 0.5)
    bottom = dataclasses.replace(col, escape_diff_limited=None, v_top=None, v_dep=v_dep)
    prob = transport_only(net, bottom)
    n_ss, _ = integrate.be_step(prob, np.zeros_like(col.n0), 1e30)
    assert np.abs(v_dep * n_ss[0] - col.phi_surf).max() <= 1e-13 * col.phi_surf.max()


def test_steady_state_carries_the_emitted_flux_out_of_the_top(net_col):
    """Emission at the bottom, escape at the top: every level carries the
    emitted flux and v_top n_{N-1} = phi_surf.  On an 8-layer column from 1
    to 0.2 bar (across the whole 120-layer column the slowest mode, escape
    seen through the top layer's tiny density, leaves the linear problem too
    ill-conditioned for an FP64 steady state)."""
    net, _ = net_col
    S, N = len(net.mass_amu), 8
    short = synth.column.Column(P_bar=np.geomspace(1.0, 0.2, N), T_K=np.full(N, 1200.0),
                                Kzz=np.full(N, 1e8), Dmol=None, alphaT=None,
                                n0=np.zeros((N, S)))
    phi = np.where(np.arange(S) % 7 == 0, 1e10, 0.0)
    v_top = np.full(S, 0.5)
    prob = transport_only(net, dataclasses.replace(short, v_top=v_top, phi_surf=phi))
    n_ss, _ = integrate.be_step(prob, short.n0, 1e30)
    assert np.abs(v_top * n_ss[-1] - phi).max() <= 1e-12 * phi.max()
    assert np.all(n_ss[:, phi == 0] == 0.0)


def test_diffusion_limited_velocity(net_col):
    net, col = net_col
    g = grid_mod.make_grid(col, net.mass_amu)
    m = np.asarray(net.mass_amu)
    T, D = col.T_K[-1], col.Dmol[-1]
    want = np.where(col.escape_diff_limited == 1,
                    np.maximum(D * (col.mbar_amu - m) * AMU * col.g_cgs / (KB * T), 0.0), 0.0)
    want = want + col.v_top
    assert np.allclose(g.v_top, want, rtol=1e-13, atol=0)
    # a heavier-than-mean species flagged for escape does not escape
    heavy = int(np.argmax(m))
    flags = np.zeros(len(m), np.int32)
    flags[heavy] = 1
    g2 = grid_mod.make_grid(dataclasses.replace(col, escape_diff_limited=flags, v_top=None),
                            net.mass_amu)
    assert g2.v_top[heavy] == 0.0 and np.all(g2.v_top == 0.0)


@pytest.mark.parametrize("layer", ["bottom", "top"])
def test_boundary_rows_of_the_step_matrix_are_the_derivative(net_col, layer):
    net, col = net_col
    prob = transport_only(net, col)
    N, S = col.n0.shape
    k = 0 if layer == "bottom" else N - 1
    dt = 1.0
    B, a, c = prob.step_matrix(col.n0, dt)
    for y in range(S):
        h = 1e-3 * col.n0[k, y] + 1.0
        up = col.n0.copy()
        dn = col.n0.copy()
        up[k, y] += h
        dn[k, y] -= h
        d = (prob.rhs(up)[k, y] - prob.rhs(dn)[k, y]) / (2 * h)
        assert B[k, y, y] == pytest.approx(1.0 / dt - d, rel=1e-8, abs=1e-20)
