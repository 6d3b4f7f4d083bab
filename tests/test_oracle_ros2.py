"""Pins of the oracle's second-order steps: the Rosenbrock step (ROS2:
Verwer, Spee, Blom and Hundsdorfer 1999; Section 2.1 lists Rosenbrock
solvers for this problem) and the linearly implicit BDF2 step.

* With the chemistry switched off the right-hand side is the linear
  transport operator L (built here by probing F with unit vectors), and one
  ROS2 step must equal the method's stability function applied to the state,
  R(dt L) n0 = (I - g dt L)^-2 (I + (1 - 2g) dt L) n0 with g = 1 + 1/sqrt 2
  (the z^2 term of the numerator vanishes for this g).  A wrong stage weight,
  the sign of the -2 k1 coupling or gamma changes R.
* L-stability: at dt far beyond every transport time scale the step lands
  on the diffusive equilibrium exp(dt L) n0, as R(-inf) = 0.
* Order: on the 12-species column with its full chemistry, against scipy's
  Radau at rtol 1e-12, halving the step divides the error by 4 (backward
  Euler by 2).
* BDF2 on the linear problem is the textbook recurrence
  (I - 2/3 dt L) n_new = 4/3 n - 1/3 n_prev (the linearisation is exact
  there); it reaches the diffusive equilibrium at huge dt; with the full
  chemistry, started by one backward-Euler step, it is second order
  against Radau."""

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import synth
from oracle import integrate


@pytest.fixture(scope="module")
def transport_only():
    net, col = synth.make_config(1)
    prob = integrate.Problem(net, col)
    prob.kf = np.zeros_like(prob.kf)
    prob.kr = np.zeros_like(prob.kr)
    N, S = col.n0.shape
    n0 = col.n0 * (1.0 + 0.5 * np.random.default_rng(3).random(col.n0.shape))
    L = np.zeros((N * S, N * S))
    for j in range(N * S):
        e = np.zeros(N * S)
        e[j] = 1.0
        L[:, j] = prob.rhs(e.reshape(N, S)).ravel()
    assert np.abs(prob.rhs(n0).ravel() - L @ n0.ravel()).max() \
        <= 1e-12 * np.abs(prob.rhs(n0)).max()
    return prob, n0, L


@pytest.mark.parametrize("dt", [1e3, 1e5, 1e7, 1e9])
def test_ros2_on_a_linear_problem_is_its_stability_function(transport_only, dt):
    prob, n0, L = transport_only
    g = 1.0 + 1.0 / np.sqrt(2.0)
    eye = np.eye(L.shape[0])
    W = eye - g * dt * L
    want = np.linalg.solve(W, np.linalg.solve(W, (eye + (1 - 2 * g) * dt * L) @ n0.ravel()))
    got, delta = integrate.ros2_step(prob, n0, dt)
    assert np.abs(got.ravel() - want).max() <= 1e-13 * np.abs(want).max()
    assert np.allclose(got - n0, delta, rtol=0, atol=1e-15 * np.abs(n0).max())


def test_ros2_local_error_is_third_order(transport_only):
    prob, n0, L = transport_only
    errs = []
    for dt in (1e3, 2e3):
        exact = expm(dt * L) @ n0.ravel()
        got, _ = integrate.ros2_step(prob, n0, dt)
        errs.append(np.abs(got.ravel() - exact).max())
    assert 6.0 < errs[1] / errs[0] < 10.0


def test_ros2_is_l_stable(transport_only):
    prob, n0, L = transport_only
    dt = 1e14
    eq = expm(dt * L) @ n0.ravel()
    got, _ = integrate.ros2_step(prob, n0, dt)
    assert np.abs(got.ravel() - eq).max() <= 1e-7 * np.abs(eq).max()
    # it moved: the perturbed state is far from that equilibrium
    assert np.abs(n0.ravel() - eq).max() > 1e-2 * np.abs(eq).max()


def test_ros2_is_second_order_on_the_chemistry():
    net, col = synth.make_config(1)
    prob = integrate.Problem(net, col)
    N, S = col.n0.shape
    T = 1e-6
    ref = solve_ivp(lambda t, y: prob.rhs(y.reshape(N, S)).ravel(), (0.0, T),
                    col.n0.ravel(), method="Radau", rtol=1e-12, atol=1e-16)
    assert ref.status == 0
    yT = ref.y[:, -1]

    def err(step, m):
        n = col.n0.copy()
        for _ in range(m):
            n, _ = step(prob, n, T / m)
        return np.abs(n.ravel() - yT).max() / np.abs(yT).max()

    r = [err(integrate.ros2_step, m) for m in (4, 8, 16)]
    assert 3.5 < r[0] / r[1] < 4.5 and 3.5 < r[1] / r[2] < 4.5
    b = [err(integrate.be_step, m) for m in (4, 8)]
    assert 1.8 < b[0] / b[1] < 2.2
    assert r[2] < 1e-2 * b[1]


@pytest.mark.parametrize("dt", [1e3, 1e6, 1e9])
def test_bdf2_on_a_linear_problem_is_the_bdf2_recurrence(transport_only, dt):
    prob, n0, L = transport_only
    n_prev = n0 * (1.0 + 0.1 * np.random.default_rng(4).random(n0.shape))
    eye = np.eye(L.shape[0])
    want = np.linalg.solve(eye - (2.0 / 3.0) * dt * L,
                           (4.0 / 3.0) * n0.ravel() - (1.0 / 3.0) * n_prev.ravel())
    got, delta = integrate.bdf2_step(prob, n0, n_prev, dt)
    assert np.abs(got.ravel() - want).max() <= 1e-12 * np.abs(want).max()
    assert np.allclose(got - n0, delta, rtol=0, atol=1e-15 * np.abs(n0).max())


def test_bdf2_reaches_the_equilibrium_at_huge_dt(transport_only):
    prob, n0, L = transport_only
    dt = 1e14
    eq = expm(dt * L) @ n0.ravel()
    n1, _ = integrate.bdf2_step(prob, n0, n0, dt)
    n2, _ = integrate.bdf2_step(prob, n1, n0, dt)
    assert np.abs(n2.ravel() - eq).max() <= 1e-6 * np.abs(eq).max()


def test_bdf2_is_second_order_on_the_chemistry():
    net, col = synth.make_config(1)
    prob = integrate.Problem(net, col)
    N, S = col.n0.shape
    T = 1e-6
    ref = solve_ivp(lambda t, y: prob.rhs(y.reshape(N, S)).ravel(), (0.0, T),
                    col.n0.ravel(), method="Radau", rtol=1e-12, atol=1e-16)
    yT = ref.y[:, -1]

    def err(m):
        h = T / m
        prev = col.n0
        n, _ = integrate.be_step(prob, prev, h)   # one O(h^2) starting step
        for _ in range(m - 1):
            n, prev = integrate.bdf2_step(prob, n, prev, h)[0], n
        return np.abs(n.ravel() - yT).max() / np.abs(yT).max()

    e = [err(m) for m in (8, 16, 32)]
    assert 3.8 < e[0] / e[1] < 4.2 and 3.8 < e[1] / e[2] < 4.2


def test_backward_euler_and_ros2_drivers_reach_the_same_steady_state():
    """The steady state is the fixed point F(n) = 0 (of the clipped
    iteration), whichever step the driver takes to reach it."""
    net, col = synth.make_config(1)
    prob = integrate.Problem(net, col)
    kw = dict(tol_rel=1e-13, t_end=1e30, max_steps=4000)
    a = integrate.steady_state(prob, col.n0, **kw)
    b = integrate.steady_state(prob, col.n0, method="ros2", **kw)
    assert a.converged and b.converged
    keep = a.n > 1e-30 * prob.grid.ngas[:, None]
    assert np.max(np.abs(a.n - b.n)[keep] / a.n[keep]) < 1e-7


@pytest.mark.parametrize("w", [0.5, 1.0, 3.0])
def test_variable_step_bdf2_on_a_linear_problem_is_the_recurrence(transport_only, w):
    """(I - b dt L) n_new = (1+w)^2/(1+2w) n - w^2/(1+2w) n_prev, b = (1+w)/(1+2w)."""
    prob, n0, L = transport_only
    dt_prev = 1e5
    dt = w * dt_prev
    n_prev = n0 * (1.0 + 0.1 * np.random.default_rng(8).random(n0.shape))
    eye = np.eye(L.shape[0])
    b = (1 + w) / (1 + 2 * w)
    want = np.linalg.solve(eye - b * dt * L, (1 + w) ** 2 / (1 + 2 * w) * n0.ravel()
                           - w * w / (1 + 2 * w) * n_prev.ravel())
    got, _ = integrate.bdf2_step(prob, n0, n_prev, dt, dt_prev)
    assert np.abs(got.ravel() - want).max() <= 1e-12 * np.abs(want).max()


def test_variable_step_bdf2_is_second_order_on_the_chemistry():
    """Steps alternating between h and 2h (ratios 2 and 1/2), halved together."""
    net, col = synth.make_config(1)
    prob = integrate.Problem(net, col)
    N, S = col.n0.shape
    T = 1e-6
    ref = solve_ivp(lambda t, y: prob.rhs(y.reshape(N, S)).ravel(), (0.0, T),
                    col.n0.ravel(), method="Radau", rtol=1e-12, atol=1e-16)
    yT = ref.y[:, -1]

    def err(m):
        steps = [T / (1.5 * m) * (1.0 if i % 2 == 0 else 2.0) for i in range(m)]
        prev = col.n0
        n, _ = integrate.be_step(prob, prev, steps[0])
        for i in range(1, m):
            n, prev = integrate.bdf2_step(prob, n, prev, steps[i], steps[i - 1])[0], n
        return np.abs(n.ravel() - yT).max() / np.abs(yT).max()

    e = [err(m) for m in (8, 16, 32)]
    assert 3.6 < e[0] / e[1] < 4.4 and 3.6 < e[1] / e[2] < 4.4
