"""GPU parity of the factor-reusing step (xod_step_frozen): backward-Euler
steps that solve with the step matrix of an earlier state, against the
oracle's frozen_step with the same matrix.  Tolerance: the per-layer
agreement of the other solve tests (rel 1e-9 covers cyclic reduction)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import integrate  # noqa: E402
from tests import gpu_common as G  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_2512_06729_amd  # noqa: F401  (fails loudly if not built)


@pytest.mark.parametrize("solver,cfg,dt", [(0, 2, 1e-6), (1, 2, 1e-6), (1, 3, 1e-7), (0, 1, 1e-3), (1, 1, 1e-3)])
def test_frozen_steps_match_oracle(solver, cfg, dt):
    import paper_2512_06729_amd as xod
    print(f"frozen solver={solver} config {cfg} dt={dt}", flush=True)
    net, col = synth.make_config(cfg)
    prob, gnet, gcol = G.make_pair(net, col)
    gcol.set_solver(solver)
    frozen = prob.step_matrix(col.n0, dt)
    n, delta = integrate.be_step(prob, col.n0, dt)
    xod.xod_step(gcol, dt)
    G.assert_state_agrees(gcol.state(), n, delta, rel=1e-9)
    for _ in range(3):
        n_ref, delta = integrate.frozen_step(prob, n, frozen)
        xod.xod_step_frozen(gcol, dt)
        got = gcol.state()
        G.assert_state_agrees(got, n_ref, delta, rel=1e-9)
        n = n_ref


def test_frozen_step_needs_a_factorisation_of_that_dt():
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(1)
    _, gnet, gcol = G.make_pair(net, col)
    with pytest.raises(xod.XodError) as e:
        xod.xod_step_frozen(gcol, 1e-6)
    assert e.value.status == xod.XOD_EINVAL
    xod.xod_step(gcol, 1e-6)
    with pytest.raises(xod.XodError) as e:
        xod.xod_step_frozen(gcol, 2e-6)
    assert e.value.status == xod.XOD_EINVAL
    xod.xod_step_frozen(gcol, 1e-6)
    gcol.set_solver(xod.XOD_SOLVER_CR)
    with pytest.raises(xod.XodError) as e:
        xod.xod_step_frozen(gcol, 1e-6)
    assert e.value.status == xod.XOD_EINVAL
