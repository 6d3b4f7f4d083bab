"""The explicit block calls through the C ABI with either factorisation and
either precision: xod_jacobian builds M = (B, a, c) on the device,
xod_btd_factor(..., precision) factors it with the column's solver and
xod_btd_solve(..., max_refine) solves M x = F(n), compared with the oracle's
block-Thomas solve of the same system.

Tolerances: the forward-error bound of a backward-stable solve, per layer
rel |x| + 10 kappa eps max_layer |x| with kappa the diagonal blocks'
condition number (rel 1e-10 for block Thomas, 1e-9 for cyclic reduction,
whose elimination combines layers far apart); mixed precision after
refinement at the same bounds, since the refined solution converges to the
FP64 system's solution (componentwise to 1e-7 of each solution entry or
1e-14 of its layer's largest)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import linalg  # noqa: E402
from tests import gpu_common as G  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_2512_06729_amd  # noqa: F401  (fails loudly if not built)


def system(gcol, prob, n0, dt):
    """Device (B, a, c) of the step matrix at n0 (xod_jacobian) and, as the
    right-hand side, the oracle's F(n0): both sides solve for the same
    vector, so the comparison measures the solves alone (F's own rounding,
    amplified by the conditioning, would otherwise dominate)."""
    kf, kr = G.gpu_rates(gcol)
    n, B, a, c = G.gpu_blocks(gcol, kf, kr, n0, dt)
    f = torch.from_numpy(np.ascontiguousarray(prob.rhs(n0))).to(G.dev()).reshape(-1)
    return B, a, c, f


@pytest.mark.parametrize("cfg,dt", [(1, 1e-6), (2, 1e-6), (2, 1e-8)])
@pytest.mark.parametrize("solver", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_factor_solve_through_the_abi(cfg, dt, solver, precision):
    import paper_2512_06729_amd as xod
    print(f"btd abi: config {cfg} dt {dt} solver {solver} precision {precision}", flush=True)
    net, col, prob, gnet, gcol = G.config_pair(cfg)
    gcol.set_solver(solver)
    B, a, c, f = system(gcol, prob, col.n0, dt)
    Bo, ao, co = prob.step_matrix(col.n0, dt)
    ref = linalg.btd(Bo, ao, co, prob.rhs(col.n0))
    B_in = B.clone()
    piv = torch.empty(gcol.N * gcol.ld, dtype=torch.int32, device=G.dev())
    xod.xod_btd_factor(gcol, B, a, c, piv, precision=precision)
    if precision == 1 or solver == 1:
        assert torch.equal(B, B_in)          # read only: the factors stay in the column
    x = f.clone()
    xod.xod_btd_solve(gcol, B, a, c, piv, x, max_refine=10)
    it, fb, size = xod.xod_btd_solve_info(gcol)
    print(f"  refinements {it}, fallback {fb}, correction size {size:.2e}")
    if precision == 1:
        assert it >= 1 and fb == 0 and size <= 10.0
    kappa = G.block_kappa(prob, col.n0, dt)
    G.assert_state_agrees_kappa(G.to_np(x, (gcol.N, gcol.S)), ref, ref, kappa,
                                rel=1e-10 if solver == 0 else 1e-9)
    # a second right-hand side with the same factors
    x2 = (2.0 * f).clone()
    xod.xod_btd_solve(gcol, B, a, c, piv, x2, max_refine=10)
    G.assert_state_agrees_kappa(G.to_np(x2, (gcol.N, gcol.S)), 2.0 * ref, 2.0 * ref, kappa,
                                rel=1e-10 if solver == 0 else 1e-9)


def test_mixed_without_refinement_and_state_checks():
    import paper_2512_06729_amd as xod
    net, col, prob, gnet, gcol = G.config_pair(2)
    gcol.set_solver(xod.XOD_SOLVER_CR)
    dt = 1e-6
    B, a, c, f = system(gcol, prob, col.n0, dt)
    Bo, ao, co = prob.step_matrix(col.n0, dt)
    ref = linalg.btd(Bo, ao, co, prob.rhs(col.n0))
    # a solve needs a factorisation of the same system first
    with pytest.raises(xod.XodError) as e:
        xod.xod_btd_solve(gcol, B, a, c, None, f.clone(), max_refine=3)
    assert e.value.status == xod.XOD_EINVAL
    xod.xod_btd_factor(gcol, B, a, c, None, precision=xod.XOD_MIXED)
    x0 = f.clone()
    xod.xod_btd_solve(gcol, B, a, c, None, x0, max_refine=0)      # the FP32 solution
    assert xod.xod_btd_solve_info(gcol)[0] == 0
    x0 = G.to_np(x0, (gcol.N, gcol.S))
    assert np.all(np.isfinite(x0))
    lm = np.abs(ref).max(axis=1, keepdims=True)
    assert np.max(np.abs(x0 - ref) / lm) < 1e-3          # FP32 accuracy, not FP64's
    # a step replaces the column's blocks: the held factorisation is gone
    xod.xod_step(gcol, dt)
    with pytest.raises(xod.XodError) as e:
        xod.xod_btd_solve(gcol, B, a, c, None, f.clone(), max_refine=3)
    assert e.value.status == xod.XOD_EINVAL
    with pytest.raises(xod.XodError) as e:
        xod.xod_btd_factor(gcol, B, a, c, None, precision=7)
    assert e.value.status == xod.XOD_EINVAL
