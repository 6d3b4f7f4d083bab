"""The persistent small-block path of block Thomas (one launch per column
for the factorisation and one for the solve, padded blocks up to 64) against
the oracle, and against the per-layer panel kernels it replaces at those
sizes (option fused_max_ld = 0).

Cases: the 12-species column (blocks padded to 32) and a 48-species,
30-layer column with molecular diffusion (blocks padded to 64), one
backward-Euler step at dt 1e-6 and 1e-2 from the initial state, held to the
forward-error bound of a backward-stable solve with the diagonal blocks'
condition number (per layer rel 1e-10 of each increment plus
10 kappa eps of the layer's largest); then a frozen step on the held
factors (the solve alone) against the oracle's frozen step."""

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
    import paper_2512_06729_amd as xod
    yield
    xod.set_option("fused_max_ld", 64)


def case(name):
    if name == "c1":
        return synth.make_config(1)
    net = synth.make_network("s48", seed=4048)
    return net, synth.make_column("c2", net, seed=4049, N=30)


@pytest.mark.parametrize("name", ["c1", "s48"])
@pytest.mark.parametrize("fused", [64, 0])
@pytest.mark.parametrize("dt", [1e-6, 1e-2])
def test_small_block_thomas_matches_oracle(name, fused, dt):
    import paper_2512_06729_amd as xod
    print(f"small-block Thomas: {name} fused_max_ld {fused} dt {dt}", flush=True)
    xod.set_option("fused_max_ld", fused)
    net, col = case(name)
    prob, gnet, gcol = G.make_pair(net, col)
    assert gcol.ld == (32 if name == "c1" else 64)
    kappa = G.block_kappa(prob, col.n0, dt)
    n_ref, delta = integrate.be_step(prob, col.n0, dt)
    xod.xod_step(gcol, dt)
    n1 = gcol.state()
    G.assert_state_agrees_kappa(n1, n_ref, delta, kappa, rel=1e-10)
    # the held factors, used by the solve alone
    frozen = prob.step_matrix(col.n0, dt)
    n_fz, d_fz = integrate.frozen_step(prob, n_ref, frozen)
    xod.xod_step_frozen(gcol, dt)
    G.assert_state_agrees_kappa(gcol.state(), n_fz, d_fz, kappa, rel=1e-10)


def test_fused_and_panel_paths_agree_over_a_schedule():
    """The 12-species column over the first 120 steps of the fixed schedule
    (dt up to 1e1 s) with both paths: the two factorisations of the same
    blocks agree to 1e-10 of each density above mixing ratio 1e-30."""
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(1)
    states = {}
    for fused in (64, 0):
        xod.set_option("fused_max_ld", fused)
        prob, gnet, gcol = G.make_pair(net, col)
        for dt in integrate.fixed_schedule(120):
            xod.xod_step(gcol, dt)
        states[fused] = gcol.state()
    ngas = prob.grid.ngas[:, None]
    keep = states[0] > 1e-30 * ngas
    err = np.max(np.abs(states[64] - states[0])[keep] / states[0][keep])
    print(f"fused vs panel after 120 steps: {err:.2e}")
    assert err <= 1e-10
