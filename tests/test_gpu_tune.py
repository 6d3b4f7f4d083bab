"""The tile-shape autotuner (xod_autotune, xod_batch_autotune): it times
its candidates on the caller's work, keeps the fastest per kind of column,
and the factorisations that then run with the tuned settings still match
the oracle (every candidate is the same factorisation up to rounding
order), at the forward-error bound with the diagonal blocks' condition
number.  The tuned table is cleared after each test."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import integrate  # noqa: E402
from tests import gpu_common as G  # noqa: E402


@pytest.fixture(autouse=True)
def _clear():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_2512_06729_amd as xod
    xod.xod_autotune_clear()
    yield
    xod.xod_autotune_clear()


@pytest.mark.parametrize("cfg,solver", [(1, 0), (1, 1), (2, 0), (2, 1)])
def test_autotune_picks_a_setting_and_steps_still_match(cfg, solver):
    import paper_2512_06729_amd as xod
    print(f"autotune: config {cfg} solver {solver}", flush=True)
    net, col, prob, gnet, gcol = G.config_pair(cfg)
    gcol.set_solver(solver)
    dt = 1e-6
    r = xod.xod_autotune(gcol, dt, trials=2)
    print(f"  {r}")
    kind = "cr" if solver == 1 else "thomas"
    assert r["key"].endswith(f"/ld{gcol.ld}/fp64/{kind}/column")
    assert r["candidates"] >= 2
    assert 0.0 < r["best_ms"] <= r["default_ms"]
    # the state did not move; a step now runs with the tuned setting
    np.testing.assert_array_equal(gcol.state(), col.n0)
    n_ref, delta = integrate.be_step(prob, col.n0, dt)
    xod.xod_step(gcol, dt)
    G.assert_state_agrees_kappa(gcol.state(), n_ref, delta, G.block_kappa(prob, col.n0, dt),
                                rel=1e-10 if solver == 0 else 1e-9)


def test_batch_autotune_per_group():
    import paper_2512_06729_amd as xod
    nets = {12: synth.make_config(1)[0], 90: synth.make_network("c2", seed=1002)}
    stream = torch.cuda.current_stream().cuda_stream
    gnets = {s: xod.Network(n) for s, n in nets.items()}
    cols, gcols, probs = [], [], []
    for j in range(6):
        s = 12 if j % 2 == 0 else 90
        col = synth.make_column("c1" if s == 12 else "c2", nets[s], seed=8100 + j,
                                N=20 if s == 12 else 40)
        cols.append(col)
        gcols.append(xod.Column(gnets[s], col, stream=stream))
        probs.append(integrate.Problem(nets[s], col))
    batch = xod.Batch(gcols)
    dts = np.full(len(gcols), 1e-6)
    res = batch.autotune(dts, trials=1)
    print(res)
    assert sorted(r["key"].split("/")[1] for r in res) == ["ld32", "ld96"]
    assert all(r["key"].endswith("/fp64/thomas/batch") for r in res)
    for g, col in zip(gcols, cols):
        np.testing.assert_array_equal(g.state(), col.n0)    # tuning does not advance
    batch.step(dts)
    for g, col, prob in zip(gcols, cols, probs):
        n_ref, delta = integrate.be_step(prob, col.n0, 1e-6)
        G.assert_state_agrees_kappa(g.state(), n_ref, delta, G.block_kappa(prob, col.n0, 1e-6))
    batch.close()


def test_autotune_argument_checks():
    import paper_2512_06729_amd as xod
    net, col, prob, gnet, gcol = G.config_pair(1)
    for dt, trials in ((0.0, 2), (1e-6, 0), (1e-6, 101)):
        with pytest.raises(xod.XodError) as e:
            xod.xod_autotune(gcol, dt, trials=trials)
        assert e.value.status == xod.XOD_EINVAL
