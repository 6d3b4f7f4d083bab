"""Pins of the oracle's modified-Newton backward-Euler step (be_step with
newton_iters > 1: corrections of the fully implicit equation
n1 - n - dt F(n1) = 0 with the step matrix of n reused, the corrector of
the DLSODES family Section 2.1 names).

* The corrections drive the residual of the implicit equation, evaluated
  here straight from its definition, down geometrically to the rounding
  floor of F.
* On the linear transport problem the linearised step is already the
  implicit solution: further corrections change nothing."""

import numpy as np
import pytest

import synth
from oracle import integrate


def residual(prob, n0, n1, dt):
    return np.abs(n1 - n0 - dt * prob.rhs(n1)).max() / np.abs(n1 - n0).max()


@pytest.mark.parametrize("cfg,dt", [(1, 1e-5), (2, 1e-6)])
def test_corrections_solve_the_implicit_equation(cfg, dt):
    net, col = synth.make_config(cfg)
    prob = integrate.Problem(net, col)
    r = [residual(prob, col.n0, integrate.be_step(prob, col.n0, dt, newton_iters=k)[0], dt)
         for k in (1, 2, 3, 4)]
    assert r[0] > 1e-4
    assert r[1] < 0.2 * r[0] and r[2] < 0.2 * r[1] and r[3] < 0.2 * r[2]
    n8, _ = integrate.be_step(prob, col.n0, dt, newton_iters=8)
    assert residual(prob, col.n0, n8, dt) < 1e-10


def test_linear_problem_needs_no_correction():
    net, col = synth.make_config(1)
    prob = integrate.Problem(net, col)
    prob.kf = np.zeros_like(prob.kf)
    prob.kr = np.zeros_like(prob.kr)
    n0 = col.n0 * (1.0 + 0.5 * np.random.default_rng(2).random(col.n0.shape))
    for dt in (1e3, 1e7):
        a, _ = integrate.be_step(prob, n0, dt)
        b, _ = integrate.be_step(prob, n0, dt, newton_iters=4)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
        assert residual(prob, n0, a, dt) < 1e-10
