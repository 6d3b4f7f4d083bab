"""Per-species error of the 594-species x 150-layer column (7720 reactions)
against the oracle over three backward-Euler steps from the initial state,
for FP64 (block cyclic reduction and block Thomas) and mixed precision (FP32
Schur complements with FP64 refinement).

Each GPU trajectory runs on its own (it is not reset to the oracle's state
between steps), so the errors are those a user of three steps sees.  The
per-species figure is the largest relative error over the layers of the
species' densities with mixing ratio above 1e-30.

Asserted: each FP64 step, against the oracle's step from the same state,
within the forward-error bound of a backward-stable solve (increments to
1e-9 relative, plus ten times the diagonal blocks' condition number times
the unit roundoff of the layer's largest increment), and mixed precision
within 1e-6 relative on every mixing ratio above 1e-30.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import integrate  # noqa: E402
from tests import gpu_common as G  # noqa: E402

DT = 1e-6
STEPS = 3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_2512_06729_amd  # noqa: F401  (fails loudly if not built)


@pytest.fixture(scope="module")
def reference():
    net, col = synth.make_config(3)
    prob = integrate.Problem(net, col)
    states, deltas = [], []
    n = col.n0
    for _ in range(STEPS):
        n, d = integrate.be_step(prob, n, DT)
        states.append(n)
        deltas.append(d)
    return net, col, prob, states, deltas


def per_species_error(n, ref, ngas):
    keep = np.abs(ref) > 1e-30 * ngas[:, None]
    rel = np.where(keep, np.abs(n - ref) / np.where(keep, np.abs(ref), 1.0), 0.0)
    return rel.max(axis=0)


@pytest.mark.parametrize("name,precision,solver", [("fp64-cr", 0, 1), ("fp64-thomas", 0, 0),
                                                   ("mixed-cr", 1, 1)])
def test_config3_three_steps_per_species(reference, name, precision, solver):
    import paper_2512_06729_amd as xod
    net, col, prob, states, deltas = reference
    print(f"config 3, {name}, {STEPS} steps of dt {DT}", flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    gcol = xod.Column(gnet, col, precision=precision, stream=stream, solver=solver)
    ngas = prob.grid.ngas
    prev = col.n0
    for i in range(STEPS):
        st = xod.xod_step(gcol, DT)
        n = gcol.state()
        err = per_species_error(n, states[i], ngas)
        worst = int(np.argmax(err))
        print(f"  step {i + 1}: max per-species rel err {err.max():.2e} (species {worst}); "
              f"species above 1e-10: {int((err > 1e-10).sum())}, above 1e-6: "
              f"{int((err > 1e-6).sum())}; refinements {st['refine_iters']}, "
              f"fallback {st['fp64_fallback']}", flush=True)
        if precision == 0:
            # the step from the GPU's own previous state, against the oracle's
            # step from the same state (the trajectory error above is the sum)
            ref_i, d_i = integrate.be_step(prob, prev, DT) if i else (states[0], deltas[0])
            G.assert_state_agrees_kappa(n, ref_i, d_i, G.block_kappa(prob, prev, DT),
                                        rel=1e-9)
        else:
            assert err.max() <= 1e-6, err.max()
        prev = n
    gcol.close()
