"""GPU parity of the spectral photolysis rates (xod_photolysis_spectral)
against the FP64 oracle (Section 2.3.3).

Tolerance: both sides sum positive terms (the optical depth over absorbers,
the rate over wavelength bins) in different orders and use different exp
implementations; the relative rounding of exp(-tau/mu) grows like tau eps,
and tau reaches a few hundred in the deepest layers.  Each rate is held to
1e-11 relative, or 1e-12 of the reaction's largest rate over the column
where it has fallen far below that (deep layers, where exp(-tau) underflows
on both sides)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import grid as grid_mod, photolysis as ph  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_2512_06729_amd  # noqa: F401  (fails loudly if not built)


def run_gpu(n, dz, absorbers, sig_ext, J0, dlam, sig_ph, t_f, mu):
    import paper_2512_06729_amd as xod
    dev = torch.device("cuda:0")
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)   # noqa: E731
    N, P, A, L = n.shape[0], sig_ph.shape[0], len(absorbers), len(J0)
    kph = torch.full((N, max(P, 1)), np.nan, dtype=torch.float64, device=dev)[:, :P].contiguous()
    work = torch.empty(xod.photolysis_workspace(N, A, L, P), dtype=torch.uint8, device=dev)
    xod.photolysis_spectral(d(n), d(dz), d(np.asarray(absorbers, np.int32)),
                            d(sig_ext.reshape(A, L)), d(J0), d(dlam), d(sig_ph), kph, work,
                            t_f=t_f, mu=mu, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return kph.cpu().numpy()


def check(g, o):
    assert np.all(np.isfinite(g))
    scale = np.abs(o).max(axis=0, keepdims=True)
    assert np.all(np.abs(g - o) <= 1e-11 * np.abs(o) + 1e-12 * scale), \
        float(np.max(np.abs(g - o) / (np.abs(o) + 1e-300)))


def test_config3_spectrum_matches_oracle():
    """150 layers x 594 species, 10,000 bins, 772 photolysis reactions, 463
    absorbers: the workload of the 594-species network."""
    net, col = synth.make_config(3)
    sp = synth.make_spectrum(net)
    dz = grid_mod.make_grid(col, net.mass_amu).dz
    args = (col.n0, dz, sp["absorbers"], sp["sig_ext"], sp["J0"], sp["dlam"], sp["sig_ph"])
    g = run_gpu(*args, t_f=0.5, mu=0.7)
    o = ph.spectral_rates(*args, t_f=0.5, mu=0.7)
    print(f"kph range {o.max():.3e} .. {o[o > 0].min():.3e}")
    check(g, o)


@pytest.mark.parametrize("N,S,A,L,P", [(1, 3, 1, 1, 1), (7, 9, 3, 37, 5), (70, 20, 0, 300, 65),
                                       (130, 40, 17, 129, 1), (3, 4, 4, 1000, 130)])
def test_ragged_sizes_match_oracle(N, S, A, L, P):
    rng = np.random.default_rng(N * 1000 + L)
    n = 10.0 ** rng.uniform(6, 12, (N, S))
    dz = rng.uniform(1e5, 1e6, N)
    absorbers = rng.choice(S, A, replace=False).astype(np.int32)
    sig_ext = 10.0 ** rng.uniform(-24, -18, (A, L))
    J0 = rng.uniform(1e10, 1e13, L)
    dlam = rng.uniform(0.5, 20, L)
    sig_ph = 10.0 ** rng.uniform(-21, -17, (P, L))
    args = (n, dz, absorbers, sig_ext, J0, dlam, sig_ph)
    check(run_gpu(*args, t_f=1.0, mu=1.0), ph.spectral_rates(*args))


def test_rejects_bad_arguments():
    import paper_2512_06729_amd as xod
    with pytest.raises(xod.XodError) as e:
        run_gpu(np.ones((2, 2)), np.ones(2), [0], np.ones((1, 3)), np.ones(3), np.ones(3),
                np.ones((1, 3)), t_f=1.0, mu=0.0)
    assert e.value.status == xod.XOD_EINVAL


@pytest.mark.parametrize("solver,dt", [(0, 1e-6), (1, 1e-6), (1, 1e-3)])
def test_step_with_lagged_spectrum_matches_oracle(solver, dt):
    """xod_step with the spectral rates of the step's starting state (2000
    bins, the 90-species network's 120 photolysis reactions) against the
    oracle's step with the same lagged rates."""
    import paper_2512_06729_amd as xod
    from oracle import integrate
    from tests import gpu_common as G
    net, col = synth.make_config(2)
    sp = synth.make_spectrum(net, L=2000)
    spec = dict(absorbers=sp["absorbers"], sig_ext=sp["sig_ext"], J0=sp["J0"], dlam=sp["dlam"],
                sig_ph=sp["sig_ph"], t_f=0.5, mu=0.7)
    prob, gnet, gcol = G.make_pair(net, col)
    gcol.set_solver(solver)
    dev = torch.device("cuda:0")
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)   # noqa: E731
    gcol.set_photolysis_spectrum(d(sp["absorbers"]), d(sp["sig_ext"]), d(sp["J0"]),
                                 d(sp["dlam"]), d(sp["sig_ph"]), t_f=0.5, mu=0.7)
    ref_prob = integrate.Problem(net, col, spectrum=spec)
    ref, delta = integrate.be_step(ref_prob, col.n0, dt)
    gray, _ = integrate.be_step(prob, col.n0, dt)
    xod.xod_step(gcol, dt)
    got = gcol.state()
    assert np.max(np.abs(ref - gray)) > 0          # the spectrum changes the step
    # the refined GPU solve is held to the oracle's own forward-error bound
    G.assert_state_agrees_kappa(got, ref, delta, G.block_kappa(ref_prob, col.n0, dt), rel=1e-9)


def test_back_to_gray_gives_the_gray_bits():
    import paper_2512_06729_amd as xod
    from tests import gpu_common as G
    net, col = synth.make_config(2)
    sp = synth.make_spectrum(net, L=500)
    dev = torch.device("cuda:0")
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)   # noqa: E731
    _, gnet, a = G.make_pair(net, col)
    b = xod.Column(gnet, col, stream=torch.cuda.current_stream().cuda_stream)
    b.set_photolysis_spectrum(d(sp["absorbers"]), d(sp["sig_ext"]), d(sp["J0"]), d(sp["dlam"]),
                              d(sp["sig_ph"]))
    xod.xod_step(b, 1e-6)
    b.set_state(col.n0)
    b.set_photolysis_spectrum()
    xod.xod_step(a, 1e-6)
    xod.xod_step(b, 1e-6)
    np.testing.assert_array_equal(a.state(), b.state())


@pytest.mark.parametrize("method", ["ros2", "bdf2"])
def test_second_order_steps_with_lagged_spectrum_match_oracle(method):
    """ROS2 and BDF2 take the spectral rates of the step's starting state for
    every stage, as the oracle's steps do."""
    import paper_2512_06729_amd as xod
    from oracle import integrate
    from tests import gpu_common as G
    net, col = synth.make_config(2)
    sp = synth.make_spectrum(net, L=2000)
    spec = dict(absorbers=sp["absorbers"], sig_ext=sp["sig_ext"], J0=sp["J0"], dlam=sp["dlam"],
                sig_ph=sp["sig_ph"], t_f=0.5, mu=0.7)
    prob, gnet, gcol = G.make_pair(net, col)
    gcol.set_solver(xod.XOD_SOLVER_CR)
    dev = torch.device("cuda:0")
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)   # noqa: E731
    gcol.set_photolysis_spectrum(d(sp["absorbers"]), d(sp["sig_ext"]), d(sp["J0"]),
                                 d(sp["dlam"]), d(sp["sig_ph"]), t_f=0.5, mu=0.7)
    ref_prob = integrate.Problem(net, col, spectrum=spec)
    dt = 1e-6
    if method == "ros2":
        ref, delta, (t1, t2) = integrate.ros2_step(ref_prob, col.n0, dt, stages=True)
        xod.xod_step_ros2(gcol, dt)
        scale = np.maximum(np.maximum(np.abs(t1), np.abs(t2)), np.abs(delta))
        G.assert_state_agrees(gcol.state(), ref, scale, rel=1e-9)
    else:
        n1, d1 = integrate.be_step(ref_prob, col.n0, dt)
        xod.xod_step(gcol, dt)
        G.assert_state_agrees(gcol.state(), n1, d1, rel=1e-9)
        ref, delta = integrate.bdf2_step(ref_prob, n1, col.n0, dt)
        xod.xod_step_bdf2(gcol, dt)
        G.assert_state_agrees(gcol.state(), ref, delta, rel=1e-9)
