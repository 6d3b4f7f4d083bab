"""GPU parity of the block cyclic-reduction factorisation (xod_column_set_solver
XOD_SOLVER_CR) against the oracle's block-Thomas / dense solves: the same
block system, eliminated in a different order.

Tolerance: cyclic reduction combines layers up to 2^l apart at level l, so
the rounding of a layer's smallest increments is relative to the magnitudes
of layers several pressure decades away, not only to its own.  The
per-layer floor of the block-Thomas tests (1e-10 x 1e-6 x the layer's
largest increment, i.e. about one unit roundoff of it) is therefore taken
ten times wider here (rel = 1e-9)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import integrate, equilibrium, linalg  # noqa: E402
from tests import gpu_common as G  # noqa: E402
from tests.helpers import balanced_c1_network  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_2512_06729_amd  # noqa: F401  (fails loudly if not built)


def cr_pair(net, col, precision=0):
    import paper_2512_06729_amd as xod
    prob, gnet, gcol = G.make_pair(net, col, precision)
    gcol.set_solver(xod.XOD_SOLVER_CR)
    return prob, gnet, gcol


# Layer counts with ragged reduction trees: 1 (root only), 2, 3, powers of
# two and their neighbours, and the 20 layers of the small configuration.
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 8, 9, 16, 17, 20])
@pytest.mark.parametrize("dt", [1e-6, 1e2])
def test_cr_step_matches_oracle_ragged(N, dt):
    """Small dt: per-layer agreement of the new state.  Large dt (the step
    matrix has cond ~1e10 here): the increment against a dense solve within
    the backward-stability bound 50 cond(M) eps, and the residual bound."""
    import paper_2512_06729_amd as xod
    print(f"cr step N={N} dt={dt}", flush=True)
    net = synth.make_network("c1", seed=1001)
    col = synth.make_column("c1", net, seed=300 + N, N=N)
    prob, gnet, gcol = cr_pair(net, col)
    st = xod.xod_step(gcol, dt)
    assert st["nonfinite"] == 0
    n = gcol.state()
    if dt <= 1e-3:
        ref, delta = integrate.be_step(prob, col.n0, dt)
        G.assert_state_agrees(n, ref, delta, rel=1e-9)
        return
    f = prob.rhs(col.n0)
    B, a, c = prob.step_matrix(col.n0, dt)
    M = linalg.assemble(B, a, c)
    ref = np.linalg.solve(M, f.ravel())
    kappa = np.linalg.cond(M)
    x = (n - col.n0).ravel()
    scale = np.abs(ref).max() + 4 * G.EPS * np.abs(n).max()
    print(f"cond {kappa:.2e} err {np.abs(x - ref).max() / (kappa * G.EPS * scale):.2e} x cond eps")
    assert np.abs(x - ref).max() <= 50 * kappa * G.EPS * scale
    r = M @ x - f.ravel()
    assert np.abs(r).max() <= 50 * kappa * G.EPS * (np.abs(M) @ np.abs(x) + np.abs(f.ravel())).max()


@pytest.mark.parametrize("cfg,dt", [(2, 1e-6), (2, 1e-8), (3, 1e-8)])
def test_cr_single_step_matches_oracle(cfg, dt):
    import paper_2512_06729_amd as xod
    print(f"cr step config {cfg} dt={dt}", flush=True)
    net, col = synth.make_config(cfg)
    prob, gnet, gcol = cr_pair(net, col)
    ref, delta = integrate.be_step(prob, col.n0, dt)
    xod.xod_step(gcol, dt)
    G.assert_state_agrees(gcol.state(), ref, delta, rel=1e-9)


def test_cr_fixed_schedule_config1_matches_oracle():
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(1)
    prob, gnet, gcol = cr_pair(net, col)
    sched = integrate.fixed_schedule(200)
    ref = integrate.run_fixed(prob, col.n0, sched)
    for dt in sched:
        assert xod.xod_step(gcol, dt)["nonfinite"] == 0
    n = gcol.state()
    keep = np.abs(ref) > 1e-30 * prob.grid.ngas[:, None]
    np.testing.assert_allclose(n[keep], ref[keep], rtol=1e-10)


def test_cr_agrees_with_thomas_config3():
    """Three steps of the 594 x 150 column, both factorisations on the GPU."""
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(3)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    gt = xod.Column(gnet, col, stream=stream)
    gc = xod.Column(gnet, col, stream=stream, solver=xod.XOD_SOLVER_CR)
    n0 = gt.state()
    for dt in (1e-7, 1e-6, 1e-5):
        xod.xod_step(gt, dt)
        xod.xod_step(gc, dt)
    a, b = gc.state(), gt.state()
    G.assert_state_agrees(a, b, b - n0, rel=1e-9)


def test_cr_closed_layer_steady_state():
    import paper_2512_06729_amd as xod
    net = balanced_c1_network()
    col = synth.make_column("c1", net, seed=77, N=3)
    col.T_K = np.array([1900.0, 1500.0, 1100.0])
    col.Kzz = np.zeros(3)
    prob, gnet, gcol = cr_pair(net, col)
    res = xod.xod_integrate_to_steady_state(gcol, tol_rel=1e-13, t_end=1e30, max_steps=4000)
    assert res["converged"] == 1
    n = gcol.state()
    A = net.elem_comp.astype(float)
    for k in range(3):
        b = A @ n[k]
        on = b > 0
        lam0 = equilibrium.initial_potentials(net.nasa7, net.t_mid, A[on], col.T_K[k], n[k])
        neq, _ = equilibrium.equilibrium_layer(net.nasa7, net.t_mid, A[on], col.T_K[k], b[on], lam0)
        keep = neq > 1e-30 * prob.grid.ngas[k]
        np.testing.assert_allclose(n[k, keep], neq[keep], rtol=1e-8)


@pytest.mark.parametrize("cfg,dt", [(1, 1e-6), (2, 1e-6), (3, 1e-7)])
def test_cr_mixed_step_matches_fp64_oracle(cfg, dt):
    import paper_2512_06729_amd as xod
    print(f"cr mixed config {cfg} dt={dt}", flush=True)
    net, col = synth.make_config(cfg)
    prob, gnet, gcol = cr_pair(net, col, precision=xod.XOD_MIXED)
    ref, delta = integrate.be_step(prob, col.n0, dt)
    st = xod.xod_step(gcol, dt)
    assert st["fp64_fallback"] == 0 and st["refine_iters"] >= 1
    n = gcol.state()
    keep = np.abs(ref) > 1e-30 * prob.grid.ngas[:, None]
    rel = np.abs(n - ref)[keep] / np.abs(ref)[keep]
    assert rel.max() <= 1e-6, rel.max()
    G.assert_state_agrees(n, ref, delta, rel=1e-8)


def test_cr_solver_switch_and_errors():
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(1)
    prob, gnet, gcol = G.make_pair(net, col)
    with pytest.raises(xod.XodError) as e:
        gcol.set_solver(7)
    assert e.value.status == xod.XOD_EINVAL
    dt = 1e-4
    gcol.set_solver(xod.XOD_SOLVER_CR)
    xod.xod_step(gcol, dt)
    a = gcol.state()
    gcol.set_state(col.n0)
    gcol.set_solver(xod.XOD_SOLVER_THOMAS)
    xod.xod_step(gcol, dt)
    b = gcol.state()
    G.assert_state_agrees(a, b, b - col.n0, rel=1e-9)


@pytest.mark.parametrize("precision", [0, 1])
def test_cr_graph_replay_matches_direct_launches(precision):
    """Captured factor / solve sequences replayed several times, with eager
    steps of another column in between, give the same bits as launching the
    kernels one by one."""
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(2)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    ga = xod.Column(gnet, col, precision=precision, stream=stream, solver=xod.XOD_SOLVER_CR)
    gb = xod.Column(gnet, col, precision=precision, stream=stream, solver=xod.XOD_SOLVER_CR)
    other = xod.Column(gnet, col, stream=stream)
    try:
        for dt in (1e-7, 1e-6, 1e-5, 1e-4):
            xod.set_option("graph", 1)
            xod.xod_step(ga, dt)
            xod.set_option("graph", 0)
            xod.xod_step(other, dt)
            xod.xod_step(gb, dt)
            np.testing.assert_array_equal(ga.state(), gb.state())
    finally:
        xod.set_option("graph", 1)


def test_update_kernels_agree():
    """The 32-column-strip trailing update (used for launches over many
    blocks: the first cyclic-reduction levels of the 594 x 150 column) gives
    the same bits as the 16-column-strip one: the same MFMA accumulation
    order per element."""
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(3)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    out = []
    try:
        for u32 in (0, 1):
            xod.set_option("update32", u32)
            g = xod.Column(gnet, col, stream=stream, solver=xod.XOD_SOLVER_CR)
            xod.xod_step(g, 1e-5)
            out.append(g.state())
            g.close()
    finally:
        xod.set_option("update32", 1)
    np.testing.assert_array_equal(out[0], out[1])


def test_block_product_tilings_agree():
    """128 x 128 and 64 x 64 product tiles, K staged 16 or 32 at a time,
    accumulate every element in the same K order: identical bits."""
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(3)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    out = []
    default_k = xod.get_option("gemm_k")
    default_lib = xod.get_option("gemm_lib")
    xod.set_option("gemm_lib", 0)
    try:
        for large, kstep in ((0, 16), (1, 16), (0, 32), (1, 32)):
            xod.set_option("gemm_large", large)
            xod.set_option("gemm_k", kstep)
            g = xod.Column(gnet, col, stream=stream, solver=xod.XOD_SOLVER_CR)
            xod.xod_step(g, 1e-5)
            out.append(g.state())
            g.close()
    finally:
        xod.set_option("gemm_large", 1)
        xod.set_option("gemm_k", default_k)
        xod.set_option("gemm_lib", default_lib)
    for o in out[1:]:
        np.testing.assert_array_equal(out[0], o)


@pytest.mark.parametrize("solver", [0, 1])
def test_outer_panel_blocking_agrees(solver):
    """Blocked Gauss-Jordan (128-column outer panels: panel updates confined
    to the outer panel, then one rank-128 update) against updating the whole
    block after every 32-column panel: the same elimination, summed in a
    different order."""
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(3)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    out = []
    n0 = None
    try:
        for outer in (32, 128):
            xod.set_option("outer", outer)
            g = xod.Column(gnet, col, stream=stream, solver=solver)
            n0 = g.state()
            xod.xod_step(g, 1e-5)
            out.append(g.state())
            g.close()
    finally:
        xod.set_option("outer", 32)
    G.assert_state_agrees(out[1], out[0], out[0] - n0, rel=1e-9)


@pytest.mark.parametrize("solver,precision", [(1, 0), (0, 0), (1, 1)])
def test_panel_exchange_variants_agree(solver, precision):
    """The pivot row exchanged after one barrier (every wave publishes its
    best row) or after two (only the winner's), and the other columns'
    eliminations deferred by one column: the same pivots and the same
    arithmetic in the same order per element, identical bits."""
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(2 if solver == 0 else 3)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    out = []
    default = (xod.get_option("panel_sync"), xod.get_option("panel_defer"))
    try:
        for sync, defer in ((1, 0), (2, 0), (2, 1)):
            xod.set_option("panel_sync", sync)
            xod.set_option("panel_defer", defer)
            g = xod.Column(gnet, col, precision=precision, stream=stream, solver=solver)
            xod.xod_step(g, 1e-5)
            out.append(g.state())
            g.close()
    finally:
        xod.set_option("panel_sync", default[0])
        xod.set_option("panel_defer", default[1])
    np.testing.assert_array_equal(out[0], out[1])
    np.testing.assert_array_equal(out[0], out[2])


@pytest.mark.parametrize("precision", [0, 1])
def test_library_block_products_match(precision):
    """Block products through rocBLAS batched GEMM (gathered operands copied
    first) against the hand-written MFMA kernel: the same products summed in
    another order, so the steps agree to rounding; and the captured graph of
    the library path replays to the same bits as its direct launches."""
    import paper_2512_06729_amd as xod
    net, col = synth.make_config(3)
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    n0 = None
    out = {}
    default = (xod.get_option("gemm_lib"), xod.get_option("graph"))
    try:
        for lib, graph in ((0, 1), (1, 0), (1, 1)):
            xod.set_option("gemm_lib", lib)
            xod.set_option("graph", graph)
            g = xod.Column(gnet, col, precision=precision, stream=stream, solver=xod.XOD_SOLVER_CR)
            n0 = g.state()
            states = []
            for dt in (1e-7, 1e-6, 1e-5):
                xod.xod_step(g, dt)
                states.append(g.state())
            out[(lib, graph)] = states
            g.close()
    finally:
        xod.set_option("gemm_lib", default[0])
        xod.set_option("graph", default[1])
    for a, b in zip(out[(1, 0)], out[(1, 1)]):
        np.testing.assert_array_equal(a, b)
    a, b = out[(1, 1)][-1], out[(0, 1)][-1]
    G.assert_state_agrees(a, b, b - n0, rel=1e-9 if precision == 0 else 1e-8)
