"""GPU parity of the transport with thermal diffusion (alpha_T in the
molecular-diffusion drift of Eq. transportflux, beta = (m_y - mbar) g /
(k_B T) + alpha_T T'/T): right-hand side, step-matrix couplings and
backward-Euler steps for both factorisations, on the 90-species column
with alpha_T drawn in [-0.4, 0.3] (negative for the light species, as for
H and He in H2)."""

import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import integrate, jacobian  # noqa: E402
from tests import gpu_common as G  # noqa: E402
from tests.test_gpu_parity import _rhs_scale  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_2512_06729_amd  # noqa: F401  (fails loudly if not built)


def thermal_pair(cfg=2):
    net, col = synth.make_config(cfg)
    rng = np.random.default_rng(17)
    alpha = rng.uniform(-0.4, 0.3, len(net.mass_amu))
    alpha[np.asarray(net.mass_amu) < col.mbar_amu] = -0.38
    tcol = dataclasses.replace(col, alphaT=alpha)
    prob, gnet, gcol = G.make_pair(net, tcol)
    return net, tcol, prob, gnet, gcol


def test_thermal_diffusion_rhs_and_couplings_match_oracle():
    import paper_2512_06729_amd as xod
    net, col, prob, gnet, gcol = thermal_pair()
    plain = integrate.Problem(net, dataclasses.replace(col, alphaT=None))
    assert np.abs(prob.rhs(col.n0) - plain.rhs(col.n0)).max() > 0   # alpha_T matters
    kf, kr = G.gpu_rates(gcol)
    n = torch.from_numpy(np.ascontiguousarray(col.n0)).to(G.dev()).reshape(-1)
    f = torch.empty_like(n)
    xod.xod_rhs(gcol, kf, kr, n, f)
    f = G.to_np(f, col.n0.shape)
    assert np.all(np.abs(f - prob.rhs(col.n0)) <= 1e-12 * _rhs_scale(prob, col.n0) + 1e-300)
    _, B, a, c = G.gpu_blocks(gcol, kf, kr, col.n0, 1e-6)
    N, S, ld = gcol.N, gcol.S, gcol.ld
    a = G.to_np(a, (N, ld))[:, :S]
    c = G.to_np(c, (N, ld))[:, :S]
    lo, di, up = jacobian.transport_coefficients(prob.grid)
    np.testing.assert_allclose(a, -lo, rtol=1e-12, atol=0)
    np.testing.assert_allclose(c, -up, rtol=1e-12, atol=0)


@pytest.mark.parametrize("solver", [0, 1])
def test_thermal_diffusion_steps_match_oracle(solver):
    import paper_2512_06729_amd as xod
    net, col, prob, gnet, gcol = thermal_pair()
    gcol.set_solver(solver)
    n = col.n0
    for i in range(2):
        ref, delta = integrate.be_step(prob, n, 1e-6)
        gcol.set_state(n, t=i * 1e-6)
        xod.xod_step(gcol, 1e-6)
        G.assert_state_agrees(gcol.state(), ref, delta, rel=1e-9)
        n = ref
