"""GPU tests of the continuous-batching server: each result is the same
alone and in the mix, admission respects the HBM budget and the slot limit,
and requests that arrive while others run are admitted as room frees up."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

import synth  # noqa: E402
from tests.helpers import balanced_c1_network  # noqa: E402


def _requests():
    net = balanced_c1_network()
    cols = []
    for i in range(5):
        col = synth.make_column("c1", net, seed=500 + i, N=3 + i)
        col.T_K = np.linspace(1900.0, 1100.0, col.N) + 25.0 * i
        col.Kzz = np.full(col.N, 1e6 * (i + 1))
        cols.append(col)
    return net, cols


@pytest.mark.parametrize("solver", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_serve_results_equal_alone_and_in_the_mix(precision, solver):
    import paper_2512_06729_amd as xod
    stream = torch.cuda.current_stream().cuda_stream
    net, cols = _requests()
    gnet = xod.Network(net)
    opts = dict(tol_rel=1e-6, t_end=1e14, max_steps=3000)
    alone = []
    for col in cols:
        c = xod.Column(gnet, col, precision=precision, stream=stream, solver=solver)
        r = xod.xod_integrate_to_steady_state(c, **opts)
        alone.append((c.state(), r))
        c.close()
    fp = xod.Server.footprint(gnet, max(c.N for c in cols), precision)
    srv = xod.Server(hbm_budget_bytes=3 * fp, max_slots=2, precision=precision, stream=stream,
                     solver=solver)
    ids = [srv.submit(gnet, cols[0], **opts), srv.submit(gnet, cols[1], **opts)]
    max_active = 0
    it = 0
    while True:
        a, q = srv.step()
        max_active = max(max_active, a)
        assert srv.usage()["used_bytes"] <= 3 * fp
        it += 1
        if it == 3:                      # arrivals while others are resident
            ids += [srv.submit(gnet, c, **opts) for c in cols[2:]]
        if a == 0 and q == 0 and it > 3:
            break
        assert it < 20000
    assert max_active <= 2
    for rid, (n_alone, r_alone) in zip(ids, alone):
        out = srv.poll(rid)
        assert out["state"] == xod.Server.DONE, out
        assert out["steps"] == r_alone["steps"] and out["rejects"] == r_alone["rejects"]
        if precision == 0:
            np.testing.assert_array_equal(out["n"], n_alone)
        else:
            keep = np.abs(n_alone) > 0
            np.testing.assert_allclose(out["n"][keep], n_alone[keep], rtol=1e-12)
        assert out["latency_s"] > 0
        srv.release(rid)
    srv.close()


def test_serve_rejects_requests_larger_than_the_budget():
    import paper_2512_06729_amd as xod
    net, cols = _requests()
    gnet = xod.Network(net)
    srv = xod.Server(hbm_budget_bytes=1024, max_slots=4)
    with pytest.raises(xod.XodError) as e:
        srv.submit(gnet, cols[0])
    assert e.value.status == xod.XOD_EINVAL
