"""GPU tests of batched steps in mixed precision: FP32 Schur complements of
every column in shared launches, refined together in FP64."""

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


def test_mixed_batch_matches_fp64_oracle():
    import paper_2512_06729_amd as xod
    stream = torch.cuda.current_stream().cuda_stream
    nets = [synth.make_network("c1", seed=1001), synth.make_network("c2", seed=1002)]
    cols_in = [(nets[0], synth.make_column("c1", nets[0], seed=21, N=20)),
               (nets[1], synth.make_column("c2", nets[1], seed=22, N=30)),
               (nets[0], synth.make_column("c1", nets[0], seed=23, N=7)),
               (nets[1], synth.make_column("c2", nets[1], seed=24, N=41))]
    gnets = [xod.Network(n) for n in nets]
    cols = [xod.Column(gnets[nets.index(net)], col, precision=xod.XOD_MIXED, stream=stream)
            for net, col in cols_in]
    batch = xod.Batch(cols)
    dts = np.array([1e-7, 1e-6, 3e-5, 1e-6])
    stats = batch.step(dts)
    for (net, col), c, dt, st in zip(cols_in, cols, dts, stats):
        prob = integrate.Problem(net, col)
        ref, delta = integrate.be_step(prob, col.n0, dt)
        n = c.state()
        keep = np.abs(ref) > 1e-30 * prob.grid.ngas[:, None]
        rel = np.abs(n - ref)[keep] / np.abs(ref)[keep]
        assert rel.max() <= 1e-6, rel.max()
        G.assert_state_agrees(n, ref, delta, rel=1e-8)
        assert st["refine_iters"] >= 1


def test_batch_rejects_mixed_precisions():
    import paper_2512_06729_amd as xod
    stream = torch.cuda.current_stream().cuda_stream
    net = synth.make_network("c1", seed=1001)
    gnet = xod.Network(net)
    a = xod.Column(gnet, synth.make_column("c1", net, seed=1, N=5), stream=stream)
    b = xod.Column(gnet, synth.make_column("c1", net, seed=2, N=5), precision=xod.XOD_MIXED,
                   stream=stream)
    with pytest.raises(xod.XodError) as e:
        xod.Batch([a, b])
    assert e.value.status == xod.XOD_EINVAL
