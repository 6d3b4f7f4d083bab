"""Pins of the oracle's integrators on kept factorisations (newton_held,
fixed_dt_reuse, steady_state_reuse: the chord / modified-Newton corrector
of the DLSODES family Section 2.1 names), against what the method fixes
independently of their own code:

* iterated to a tight tolerance, the corrections on a matrix factored at
  another state solve the implicit backward-Euler equation
  n1 - n - dt F(n1) = 0, its residual evaluated here from the definition;
* on the linear A <=> B layer the step matrix does not depend on the state,
  so one factorisation serves every step and each step is the
  backward-Euler recurrence n_A - n_eq -> (n_A - n_eq) / (1 + (k_f + k_r) dt)
  in closed form;
* the driver on kept factorisations relaxes closed layers to the
  equilibrium of an independent element-potential solve, as the plain
  driver does.
"""

import numpy as np
import pytest

import synth
from oracle import equilibrium, integrate
from oracle.linalg import btd_factor
from tests.helpers import ab_network, balanced_c1_network, simple_column


def implicit_residual(prob, n0, n1, dt):
    return np.abs(n1 - n0 - dt * prob.rhs(n1)).max() / np.abs(n1 - n0).max()


@pytest.mark.parametrize("cfg,dt", [(1, 1e-6), (2, 1e-7)])
def test_corrections_on_a_held_matrix_solve_the_implicit_equation(cfg, dt):
    net, col = synth.make_config(cfg)
    prob = integrate.Problem(net, col)
    n_f = col.n0
    n, _ = integrate.be_step(prob, n_f, dt)          # the state has moved on
    B, a, c = prob.step_matrix(n_f, dt)              # the matrix has not
    held = (btd_factor(B, a, c), a, c)
    delta, ok, it = integrate.newton_held(prob, n, dt, held, newton_tol=1e-13, max_newton=40)
    assert ok and it >= 2
    assert implicit_residual(prob, n, n + delta, dt) < 1e-9     # the rounding floor of F
    # the first correction alone is the linearised step on the stale matrix:
    # not a solution yet
    d1, _, _ = integrate.newton_held(prob, n, dt, held, newton_tol=1e-13, max_newton=1)
    assert implicit_residual(prob, n, n + d1, dt) > 1e3 * implicit_residual(prob, n, n + delta, dt)


def test_linear_layer_keeps_one_factorisation_and_follows_the_recurrence():
    net = ab_network()
    col = simple_column(1, 2, T=1300.0, n0=[[1e12, 3e10]])
    prob = integrate.Problem(net, col)
    kf, kr = prob.kf[0, 0], prob.kr[0, 0]
    tot = 1e12 + 3e10
    neq = tot * kr / (kf + kr)
    dt = 0.37 / (kf + kr)
    for m in (1, 2, 5, 12):
        n, nfact, ncorr = integrate.fixed_dt_reuse(prob, col.n0, dt, m)
        expect = neq + (1e12 - neq) / (1 + (kf + kr) * dt) ** m
        assert n[0, 0] == pytest.approx(expect, rel=1e-12)
        assert n[0].sum() == pytest.approx(tot, rel=1e-14)
        assert nfact == 1
        # each step after the first: the full step, then a vanishing correction
        assert ncorr == 2 * (m - 1)


def test_reuse_driver_relaxes_closed_layers_to_element_potential_equilibrium():
    net = balanced_c1_network()
    T = np.array([1900.0, 1500.0, 1100.0])
    col = synth.make_column("c1", net, seed=77, N=3)
    col.T_K = T
    col.Kzz = np.zeros(3)
    prob = integrate.Problem(net, col)
    res = integrate.steady_state_reuse(prob, col.n0, tol_rel=1e-13, t_end=1e30, max_steps=4000)
    assert res.converged
    assert res.factorizations < res.steps          # factorisations were kept
    A = net.elem_comp.astype(float)
    for k in range(3):
        b = A @ res.n[k]
        on = b > 0
        lam0 = equilibrium.initial_potentials(net.nasa7, net.t_mid, A[on], T[k], col.n0[k])
        neq, _ = equilibrium.equilibrium_layer(net.nasa7, net.t_mid, A[on], T[k], b[on], lam0)
        keep = neq > 1e-30 * prob.grid.ngas[k]
        np.testing.assert_allclose(res.n[k, keep], neq[keep], rtol=1e-6)
