"""Pins of the oracle's Lagrangian parcel scheme (Section 2 parcel figure,
Section 2.1 molecular diffusion as a pseudo-reaction), checked against what
the method fixes independently of its own formulas:

* with molecular diffusion off the parcel carries its element content
  unchanged from layer to layer (chemistry conserves elements, the move
  keeps mixing ratios), and a parcel at the element-potential equilibrium
  of its layer (an independent Gibbs-minimum solve) stays there;
* with chemistry off, a parcel holding the density of a profile in the
  discrete diffusive equilibrium y_{k+1}/y_k = (D/dzh - D beta/2) /
  (D/dzh + D beta/2) is not moved by the pseudo-reaction, and one off it
  is;
* a visit of a single reversible A <=> B layer is the backward-Euler
  recurrence n_A - n_eq = (n_A0 - n_eq) / (1 + (k_f + k_r) dt)^m in closed
  form;
* the path goes bottom, up to the top once, and back to the bottom.
"""

import numpy as np
import pytest

import synth
from oracle import equilibrium, integrate, parcel
from tests.helpers import ab_network, balanced_c1_network, simple_column


def test_path_bottom_top_bottom():
    assert parcel.path(4) == [0, 1, 2, 3, 2, 1, 0]
    assert parcel.path(1) == [0]


def test_parcel_carries_its_element_content_without_diffusion():
    """Chemistry alone conserves elements, and the parcel keeps its mixing
    ratios from layer to layer: the element mixing ratios A p / n_gas leave
    every layer as they arrived (up to clipped negatives)."""
    net = balanced_c1_network()
    col = synth.make_column("c1", net, seed=78, N=6)
    prob = integrate.Problem(net, col)
    diff = parcel.diffusion_coefficients(prob.grid)
    assert all(np.all(d == 0) for d in diff)       # config-1 family: no molecular diffusion
    t_res = parcel.residence_times(col, prob.grid)
    A = net.elem_comp.astype(float)
    ngas = prob.grid.ngas
    seq = parcel.path(prob.grid.N)
    p = col.n0[seq[0]].copy()
    e0 = A @ p / ngas[seq[0]]
    dt = 1e-8
    clipped = 0.0
    for i, k in enumerate(seq):
        if i > 0:
            p = p * (ngas[k] / ngas[seq[i - 1]])
        q, dt, _, _, cl = parcel.visit(prob, k, p, col.n0, diff, t_res[k], min(dt, t_res[k]))
        clipped += cl / ngas[k]
        # elements change only through clipped negatives
        # (to the rounding of steps up to dt ~ 1e7 s, amplified along the
        # conserved directions as in the column's conservation test)
        assert np.all(np.abs(A @ q / ngas[k] - e0) <= clipped * A.max() + 1e-9 * e0.max())
        p = q


def test_equilibrium_parcel_stays_at_equilibrium():
    """A parcel arriving at the element-potential equilibrium of its layer
    (an independent Gibbs-minimum solve) leaves it unchanged: every
    reaction is in detailed balance, so F = 0 and the visit's steps are
    zero to rounding."""
    net = balanced_c1_network()
    T = 1700.0
    col = simple_column(1, net.nasa7.shape[0], T=T, P_bot=1.0, P_top=1.0)
    col.P_bar = np.array([1.0])
    prob = integrate.Problem(net, col)
    A = net.elem_comp.astype(float)
    ngas = prob.grid.ngas[0]
    y0 = synth.make_column("c1", net, seed=5, N=1).n0[0]
    y0 = y0 / y0.sum()
    b = A @ (y0 * ngas)
    on = b > 0
    lam0 = equilibrium.initial_potentials(net.nasa7, net.t_mid, A[on], T, y0 * ngas)
    neq, _ = equilibrium.equilibrium_layer(net.nasa7, net.t_mid, A[on], T, b[on], lam0)
    diff = parcel.diffusion_coefficients(prob.grid)
    for t_res in (1e-6, 1.0, 1e6):
        p = parcel.visit(prob, 0, neq.copy(), neq[None, :], diff, t_res, 1e-8)[0]
        keep = neq > 1e-30 * ngas
        np.testing.assert_allclose(p[keep], neq[keep], rtol=1e-8)
    # and a parcel away from equilibrium does move
    off = neq * np.where(np.arange(neq.shape[0]) % 2, 1.5, 0.7)
    p = parcel.visit(prob, 0, off, off[None, :], diff, 1.0, 1e-8)[0]
    assert np.max(np.abs(p / off - 1.0)) > 1e-3


def diffusion_only_problem(N=6, S=3):
    """Three inert species of different masses, molecular diffusion only."""
    from synth.network import small_network
    from tests.helpers import nasa_from_g
    net = small_network([[1], [1], [1]], ["X"], [], nasa_from_g([0.0, 0.0, 0.0]),
                        mass_amu=[2.0, 2.3, 5.0])
    P = np.logspace(-1, -4, N)
    T = np.linspace(1500.0, 1100.0, N)
    ngas = P * 1e6 / (1.380649e-16 * T)
    D = 1e21 * (T[:, None] / 1000.0) ** 0.7 / ngas[:, None] * np.ones((N, S))
    col = simple_column(N, S, P_bot=P[0], P_top=P[-1], T_profile=T, Kzz=1e8, D=D,
                        n0=np.ones((N, S)))
    col.P_bar = P
    return net, col


def test_diffusive_equilibrium_profile_is_a_fixed_point_of_the_visits():
    """Chemistry off: at a profile in the discrete diffusive equilibrium
    y_{k+1}/y_k = (D/dzh - D beta/2) / (D/dzh + D beta/2) (K = 0), a parcel
    holding the profile's density at its layer is not moved by the
    pseudo-reaction (the transport terms vanish there); a parcel off the
    profile is moved."""
    net, col = diffusion_only_problem()
    prob = integrate.Problem(net, col)
    g = prob.grid
    y = np.ones((g.N, g.S))
    for k in range(g.N - 1):
        half = 0.5 * g.Dh[k] * g.beta[k]
        up = g.Dh[k] / g.dzh[k]
        y[k + 1] = y[k] * (up - half) / (up + half)
    prof0 = y * 1e-3 * g.ngas[:, None]
    assert np.all(prof0 > 0)
    diff = parcel.diffusion_coefficients(g)
    for k in range(g.N):
        p = parcel.visit(prob, k, prof0[k].copy(), prof0, diff, 1e9, 1e3)[0]
        np.testing.assert_allclose(p, prof0[k], rtol=1e-9)
    k = 2
    p = parcel.visit(prob, k, 1.3 * prof0[k], prof0, diff, 1e9, 1e3)[0]
    assert np.max(np.abs(p / (1.3 * prof0[k]) - 1.0)) > 1e-3


def test_visit_of_a_linear_layer_is_the_backward_euler_recurrence():
    """A <=> B: every step of the visit is the backward-Euler map of the
    linear ODE, n_A - n_eq -> (n_A - n_eq) / (1 + (k_f + k_r) h), so the
    visit's result is the product over its step sizes h_j, in closed form."""
    net = ab_network()
    col = simple_column(1, 2, T=1500.0, n0=np.array([[3.0e12, 1.0e11]]))
    prob = integrate.Problem(net, col)
    kf, kr = prob.kf[0, 0], prob.kr[0, 0]
    diff = parcel.diffusion_coefficients(prob.grid)
    lam = kf + kr
    t_res = 7.0 / lam
    p, dt_next, steps, rejects, clipped = parcel.visit(prob, 0, col.n0[0].copy(), col.n0,
                                                       diff, t_res, 0.01 / lam)
    assert rejects == 0 and clipped == 0.0 and steps >= 3
    # the step sizes the control takes: doubling while c < 0.5, the last one
    # cut at t_res; reproduce them from the closed form of each step
    tot = col.n0[0].sum()
    a_eq = kr * tot / lam
    a, t, h = col.n0[0, 0], 0.0, 0.01 / lam
    while t < t_res:
        h = min(h, t_res - t)
        a_new = a_eq + (a - a_eq) / (1.0 + lam * h)
        c = abs(a_new - a) / max(a_new, a)
        c = max(c, abs((tot - a_new) - (tot - a)) / max(tot - a_new, tot - a))
        t += h
        a = a_new
        h = h * (2.0 if c < 0.5 else (1.2 if c < 0.9 else 0.7))
    np.testing.assert_allclose(p, [a, tot - a], rtol=1e-12)
