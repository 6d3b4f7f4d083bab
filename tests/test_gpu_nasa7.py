"""GPU parity of the Gibbs energies and rate coefficients with real two-range
NASA-7 sets (Appendix A: a2..a5 nonzero, low and high ranges distinct), on
layers below, exactly at and above the range switch at t_mid = 1000 K.

The seven coefficient pairs printed in the paper's Appendix A table are the
species.  The reactions are chosen so that each species' G/RT can be read
back from the GPU's reverse rates alone:

  X_0 <=> (nothing)   k_r/k_f = exp(-g_0 + ln(P0/kT))        (dnu = -1)
  X_y <=> X_0         k_r/k_f = exp(g_0 - g_y)                (dnu = 0)

plus two-body and three-body reactions between the species (Kooij and
modified Arrhenius), which exercise the polynomial inside the full rate
kernel.  Tolerance: 1e-12 relative on k_f and k_r, and 1e-11 absolute on
G/RT read back through a logarithm of a ratio of two rounded rates."""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import integrate, thermo  # noqa: E402
from oracle.constants import KB, P_STD  # noqa: E402
from synth.network import small_network  # noqa: E402
from tests import gpu_common as G  # noqa: E402
from tests.helpers import simple_column  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "nasa7_table.txt")

# Temperatures (bottom to top): both sides of the switch, the switch itself
# (the high range applies at T = t_mid) and the edges of the table's ranges.
T_LAYERS = [2900.0, 1600.0, 1000.5, 1000.0, 999.5, 700.0, 350.0]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_2512_06729_amd  # noqa: F401  (fails loudly if not built)


def table_sets():
    names, sets = [], {}
    with open(GOLDEN) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            p = ln.split()
            sets.setdefault(p[0], {})[p[1]] = [float(x) for x in p[2:9]]
            if p[0] not in names:
                names.append(p[0])
    return names, np.array([[sets[n]["low"], sets[n]["high"]] for n in names])


def network():
    names, nasa = table_sets()
    S = len(names)
    comp = np.eye(S, dtype=np.int32)[:, :1] + 1       # compositions are diagnostics only
    rx = [dict(type="bi", reac=[0], prod=[], params=[np.log(3e-3), 0.3, 200.0])]
    for y in range(1, S):
        rx.append(dict(type="bi", reac=[y], prod=[0],
                       params=[np.log(1e-2 / y), -0.5 + 0.2 * y, 100.0 * y],
                       kooij=bool(y % 2)))
    rx += [dict(type="bi", reac=[1, 2], prod=[3, 4], params=[np.log(2e-11), 0.7, 900.0]),
           dict(type="bi", reac=[5, 5], prod=[6, 0], params=[np.log(4e-12), -1.1, 50.0],
                kooij=True),
           dict(type="ter", reac=[2, 3], prod=[6],
                params=[np.log(1e-31), -1.5, 300.0, np.log(1e-11), 0.2, 100.0])]
    return small_network(comp, ["X"], rx, nasa, mass_amu=np.linspace(18.0, 62.0, S)), names


def test_two_range_gibbs_and_rates_match_oracle():
    import paper_2512_06729_amd as xod
    net, names = network()
    S, N = net.nasa7.shape[0], len(T_LAYERS)
    col = simple_column(N, S, T_profile=T_LAYERS, P_bot=1e1, P_top=1e-3,
                        n0=np.full((N, S), 1e10))
    prob, gnet, gcol = G.make_pair(net, col)
    kf, kr = G.gpu_rates(gcol)
    R = net.rtype.shape[0]
    kf, kr = G.to_np(kf, (N, R)), G.to_np(kr, (N, R))
    np.testing.assert_allclose(kf, prob.kf, rtol=1e-12, atol=0)
    np.testing.assert_allclose(kr, prob.kr, rtol=1e-12, atol=0)

    # G/RT of every species on every layer, read back from the GPU's rates
    # and compared with the Appendix A polynomial of the range that applies
    lnpref = np.log(P_STD / (KB * np.asarray(T_LAYERS)))
    g0 = -np.log(kr[:, 0] / kf[:, 0]) + lnpref
    g = np.empty((N, S))
    g[:, 0] = g0
    for y in range(1, S):
        g[:, y] = g0 - np.log(kr[:, y] / kf[:, y])
    for k, T in enumerate(T_LAYERS):
        rng = 1 if T >= 1000.0 else 0
        expect = np.array([thermo.g_over_rt(net.nasa7[y, rng], T) for y in range(S)])
        np.testing.assert_allclose(g[k], expect, rtol=0, atol=1e-11)
        # the other range differs by far more than the tolerance, so a switch
        # at the wrong side of t_mid (or a missing T^n term) cannot pass
        other = np.array([thermo.g_over_rt(net.nasa7[y, 1 - rng], T) for y in range(S)])
        assert np.max(np.abs(other - expect)) > 1e-6


def two_range_config1():
    """Config 1's network with every species given two distinct ranges:
    its single-range (a1, a6, a7) plus seeded a2..a5 terms of O(0.1-1) in
    G/RT near 1000 K, drawn separately for each range; the column's
    temperatures run from 1300 K to 800 K through exactly 1000 K."""
    import synth
    net, col = synth.make_config(1)
    rng = np.random.default_rng(1234)
    S = net.nasa7.shape[0]
    nasa = net.nasa7.copy()
    scale = np.array([1e-3, 1e-6, 1e-9, 1e-12])
    for r in range(2):
        nasa[:, r, 1:5] = rng.uniform(-1.0, 1.0, (S, 4)) * scale
    net.nasa7 = nasa
    N = col.N
    logp = np.log10(col.P_bar)
    T = 1300.0 - 500.0 * (logp[0] - logp) / (logp[0] - logp[-1])
    T[np.argmin(np.abs(T - 1000.0))] = 1000.0
    col.T_K = T
    from synth.column import _number_density
    y0 = col.n0 / _number_density(col.P_bar, np.linspace(2000.0, 1000.0, N))[:, None]
    col.n0 = np.ascontiguousarray(y0 * _number_density(col.P_bar, T)[:, None])
    return net, col


def test_two_range_step_matches_oracle():
    """Rates and one backward-Euler step of config 1 with two-range NASA-7
    sets on a column crossing t_mid (rates, right-hand side, Jacobian,
    factorisation, solve), for both factorisations."""
    import paper_2512_06729_amd as xod
    net, col = two_range_config1()
    assert np.any(col.T_K == 1000.0) and col.T_K.min() < 1000.0 < col.T_K.max()
    prob, gnet, gcol = G.make_pair(net, col)
    N, R = col.N, net.rtype.shape[0]
    kf, kr = G.gpu_rates(gcol)
    np.testing.assert_allclose(G.to_np(kf, (N, R)), prob.kf, rtol=1e-12, atol=0)
    np.testing.assert_allclose(G.to_np(kr, (N, R)), prob.kr, rtol=1e-12, atol=0)
    for solver in (xod.XOD_SOLVER_THOMAS, xod.XOD_SOLVER_CR):
        gcol.set_solver(solver)
        for dt in (1e-6, 1e-2):
            gcol.set_state(col.n0)
            n_ref, delta = integrate.be_step(prob, col.n0, dt)
            xod.xod_step(gcol, dt)
            # the forward-error bound of a backward-stable solve, with the
            # diagonal blocks' condition number (components 1e-10 of their
            # layer's largest increment sit at that floor)
            G.assert_state_agrees_kappa(gcol.state(), n_ref, delta,
                                        G.block_kappa(prob, col.n0, dt),
                                        rel=1e-10 if solver == xod.XOD_SOLVER_THOMAS else 1e-9)
