"""Pins for the oracle's chemistry RHS, Jacobian, linear solves and BE step
(CPU only)."""

import numpy as np
import pytest

import synth
from oracle import grid as grid_mod, rates, rhs as rhs_mod, jacobian, linalg, integrate, equilibrium
from synth.network import small_network
from tests.helpers import simple_column, nasa_from_g, ab_network, balanced_c1_network


def _random_state(prob, rng, lo=-12, hi=-1):
    g = prob.grid
    return g.ngas[:, None] * 10.0 ** rng.uniform(lo, hi, (g.N, prob.net.S))


@pytest.mark.parametrize("cfg", [1, 2])
def test_chemistry_conserves_elements(cfg):
    net, col = synth.make_config(cfg)
    prob = integrate.Problem(net, col)
    rng = np.random.default_rng(11)
    n = _random_state(prob, rng)
    w = rhs_mod.reaction_rates(net, prob.kf, prob.kr, n)
    f = rhs_mod.chem_rhs(net, w, net.S)
    A = net.elem_comp.astype(float)
    scale = np.abs(w).sum(axis=1)[:, None] * A.sum(axis=1)[None, :] * 3
    assert np.all(np.abs(f @ A.T) <= 1e-13 * scale)


def test_hand_networks_rhs():
    # A + B <=> C + D and 2 E -> F (a repeated reactant enters squared)
    comp = [[1, 0], [0, 1], [1, 0], [0, 1], [1, 1], [2, 2]]
    rx = [dict(type="bi", reac=[0, 1], prod=[2, 3], params=[np.log(1e-11), 0, 0]),
          dict(type="bi", reac=[4, 4], prod=[5], params=[np.log(2e-12), 0, 0], reversible=False)]
    net = small_network(comp, ["X", "Y"], rx, nasa_from_g([0.0, 0.0, -300.0, 200.0, 0.0, 0.0]))
    col = simple_column(1, 6, T=1000.0)
    g = grid_mod.make_grid(col, net.mass_amu)
    kf, kr = rates.rates(net, g)
    n = np.array([[3e10, 5e11, 7e9, 2e12, 4e10, 1e3]])
    f = rhs_mod.chem_rhs(net, rhs_mod.reaction_rates(net, kf, kr, n), 6)
    w1 = kf[0, 0] * n[0, 0] * n[0, 1] - kr[0, 0] * n[0, 2] * n[0, 3]
    w2 = kf[0, 1] * n[0, 4] ** 2
    expect = np.array([-w1, -w1, w1, w1, -2 * w2, w2])
    np.testing.assert_allclose(f[0], expect, rtol=1e-14)
    assert kf[0, 0] / kr[0, 0] == pytest.approx(np.exp(-(-300.0 + 200.0) / 1000.0), rel=1e-14)


@pytest.mark.parametrize("cfg", [1, 2])
def test_chemistry_jacobian_matches_central_differences(cfg):
    # f is at most quadratic in n (<= 2 reactants and <= 2 products, fixed M),
    # so central differences are exact up to rounding.
    net, col = synth.make_config(cfg)
    prob = integrate.Problem(net, col)
    rng = np.random.default_rng(7)
    n = _random_state(prob, rng, -8, -1)
    layers = [0, col.N // 2, col.N - 1]
    J = jacobian.chem_jacobian(net, prob.kf[layers], prob.kr[layers], n[layers])
    for li, k in enumerate(layers):
        for x in rng.choice(net.S, size=min(net.S, 12), replace=False):
            h = 0.1 * n[k, x]   # large h: exact for quadratics, small rounding
            npl, nmi = n[[k]].copy(), n[[k]].copy()
            npl[0, x] += h
            nmi[0, x] -= h
            fp = rhs_mod.chem_rhs(net, rhs_mod.reaction_rates(net, prob.kf[[k]], prob.kr[[k]], npl), net.S)
            fm = rhs_mod.chem_rhs(net, rhs_mod.reaction_rates(net, prob.kf[[k]], prob.kr[[k]], nmi), net.S)
            fd = (fp - fm)[0] / (2 * h)
            w = np.abs(rhs_mod.reaction_rates(net, prob.kf[[k]], prob.kr[[k]], n[[k]])).max()
            tol = 1e-9 * np.abs(J[li, :, x]) + 1e-13 * w / n[k, x]
            assert np.all(np.abs(fd - J[li, :, x]) <= tol)


def test_block_thomas_equals_dense_lu_on_tiny_columns():
    rng = np.random.default_rng(2)
    N, S = 5, 4
    B = rng.normal(size=(N, S, S)) + 3 * np.eye(S)
    a = rng.normal(size=(N, S))
    c = rng.normal(size=(N, S))
    a[0] = 0
    c[-1] = 0
    rhs = rng.normal(size=(N, S))
    np.testing.assert_allclose(linalg.btd(B, a, c, rhs), linalg.dense_solve(B, a, c, rhs), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("dt", [1e-6, 1e2, 1e6])
def test_block_thomas_equals_dense_on_config1_step_matrix(dt):
    # Both solves are backward stable, so they agree to about cond(M) * eps
    # (the step matrix grows ill-conditioned as dt grows), and each leaves a
    # residual of a few eps * |M| |x|.
    net, col = synth.make_config(1)
    prob = integrate.Problem(net, col)
    B, a, c = prob.step_matrix(col.n0, dt)
    f = prob.rhs(col.n0)
    x1 = linalg.btd(B, a, c, f)
    x2 = linalg.dense_solve(B, a, c, f)
    M = linalg.assemble(B, a, c)
    kappa = np.linalg.cond(M)
    eps = np.finfo(float).eps
    assert np.abs(x1 - x2).max() <= 50 * kappa * eps * np.abs(x2).max()
    r = M @ x1.ravel() - f.ravel()
    assert np.abs(r).max() <= 50 * eps * (np.abs(M).sum(axis=1).max() * np.abs(x1).max())


def test_block_thomas_without_transport_splits_into_layers():
    rng = np.random.default_rng(4)
    N, S = 4, 6
    B = rng.normal(size=(N, S, S)) + 2 * np.eye(S)
    z = np.zeros((N, S))
    rhs = rng.normal(size=(N, S))
    x = linalg.btd(B, z, z, rhs)
    for k in range(N):
        np.testing.assert_allclose(x[k], np.linalg.solve(B[k], rhs[k]), rtol=1e-12)


def test_backward_euler_a_b_isomerisation_closed_form():
    # A <=> B in one closed layer: BE gives n_A^m - n_eq = (n_A^0 - n_eq)/(1+(kf+kr)dt)^m.
    net = ab_network()
    col = simple_column(1, 2, T=1300.0, n0=[[1e12, 3e10]])
    prob = integrate.Problem(net, col)
    kf, kr = prob.kf[0, 0], prob.kr[0, 0]
    tot = 1e12 + 3e10
    neq = tot * kr / (kf + kr)
    n = col.n0.copy()
    dt = 0.37 / (kf + kr)
    for m in range(1, 9):
        n, _ = integrate.be_step(prob, n, dt)
        expect = neq + (1e12 - neq) / (1 + (kf + kr) * dt) ** m
        assert n[0, 0] == pytest.approx(expect, rel=1e-12)
        assert n[0].sum() == pytest.approx(tot, rel=1e-15)


def test_element_conservation_over_fixed_schedule():
    net, col = synth.make_config(1)
    prob = integrate.Problem(net, col)
    A = net.elem_comp.astype(float)
    dz = prob.grid.dz

    def totals(n):
        return (dz[:, None] * (n @ A.T)).sum(axis=0)

    b0 = totals(col.n0)
    on = b0 > 0
    n = col.n0.copy()
    for dt in integrate.fixed_schedule(200):
        n, _ = integrate.be_step(prob, n, dt)
        if dt <= 1e4:
            assert np.all(np.abs(totals(n)[on] / b0[on] - 1) <= 1e-12)


def test_steady_state_of_closed_layers_is_element_potential_equilibrium():
    # Kzz = 0, no photolysis, every reaction reversible through Gibbs energies:
    # the kinetic steady state must be the equilibrium of an independent
    # element-potential solve (and detailed balance must hold reaction by
    # reaction).
    net = balanced_c1_network()
    T = np.array([1900.0, 1500.0, 1100.0])
    col = synth.make_column("c1", net, seed=77, N=3)
    col.T_K = T
    col.Kzz = np.zeros(3)
    prob = integrate.Problem(net, col)
    res = integrate.steady_state(prob, col.n0, tol_rel=1e-13, t_end=1e30, max_steps=4000)
    assert res.converged
    A = net.elem_comp.astype(float)
    # Element totals change only through clipping of negative densities.
    drift = np.abs(res.n @ A.T - col.n0 @ A.T)
    assert np.all(drift <= res.clipped * A.max() + 1e-12 * (col.n0 @ A.T))
    for k in range(3):
        b = A @ res.n[k]
        on = b > 0
        lam0 = equilibrium.initial_potentials(net.nasa7, net.t_mid, A[on], T[k], col.n0[k])
        neq, _ = equilibrium.equilibrium_layer(net.nasa7, net.t_mid, A[on], T[k], b[on], lam0)
        keep = neq > 1e-30 * prob.grid.ngas[k]
        np.testing.assert_allclose(res.n[k, keep], neq[keep], rtol=1e-6)
        fwd = prob.kf[k] * np.prod([np.where(net.reac[:, j] >= 0, res.n[k, net.reac[:, j]], 1.0) for j in range(3)], axis=0)
        rev = prob.kr[k] * np.prod([np.where(net.prod[:, j] >= 0, res.n[k, net.prod[:, j]], 1.0) for j in range(3)], axis=0)
        big = fwd > 1e-300
        np.testing.assert_allclose(rev[big] / fwd[big], 1.0, rtol=1e-5)


def test_frozen_step_with_the_current_matrix_is_the_be_step():
    """With the matrix of the current state, the frozen step is the
    backward-Euler step; repeated frozen steps at a fixed point stay there."""
    import synth
    from oracle import integrate
    net = synth.make_network("c1", seed=1001)
    col = synth.make_column("c1", net, seed=305, N=5)
    prob = integrate.Problem(net, col)
    n0 = col.n0
    dt = 1e-4
    ref, _ = integrate.be_step(prob, n0, dt)
    got, _ = integrate.frozen_step(prob, n0, prob.step_matrix(n0, dt))
    np.testing.assert_array_equal(got, ref)
