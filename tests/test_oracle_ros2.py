"""Pins of the oracle's Rosenbrock step (ROS2: Verwer, Spee, Blom and
Hundsdorfer 1999; Section 2.1 lists Rosenbrock solvers for this problem).

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
  Euler by 2)."""

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
