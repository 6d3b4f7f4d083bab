"""Pins of the spectral photolysis oracle (Section 2.3.3): closed forms and
invariants that a dropped term, a wrong sign or index, or a transposed
operand would break."""

import numpy as np

from oracle import photolysis as ph
from oracle import rates


def test_column_density_uniform_column_closed_form():
    # uniform density n and thickness d: N(k) = n d (N - k - 1/2)
    N, n, d = 7, 3.0e10, 2.0e5
    ncol = ph.column_density(np.full((N, 1), n), np.full(N, d))
    k = np.arange(N)
    np.testing.assert_allclose(ncol[:, 0], n * d * (N - k - 0.5), rtol=1e-15)


def test_column_density_top_layer_and_monotone():
    rng = np.random.default_rng(1)
    n = rng.uniform(1, 2, (9, 3))
    dz = rng.uniform(1, 2, 9)
    ncol = ph.column_density(n, dz)
    np.testing.assert_allclose(ncol[-1], 0.5 * n[-1] * dz[-1], rtol=1e-15)
    assert np.all(np.diff(ncol, axis=0) < 0)      # more column below


def test_optically_thin_box_bands():
    # no extinction, flat J0, box cross sections: k = t_f J0 c (width)
    L = 200
    lam = np.arange(L) * 1.0
    dlam = np.ones(L)
    J0 = np.full(L, 4.0e12)
    sig_ph = np.zeros((2, L))
    sig_ph[0, 50:80] = 2.0e-18          # 30 A wide
    sig_ph[1, 10:11] = 5.0e-17          # one bin
    n = np.ones((4, 3))
    k = ph.spectral_rates(n, np.ones(4), [0, 2], np.zeros((2, L)), J0, dlam, sig_ph, t_f=0.5)
    np.testing.assert_allclose(k[:, 0], 0.5 * 4.0e12 * 2.0e-18 * 30, rtol=1e-14)
    np.testing.assert_allclose(k[:, 1], 0.5 * 4.0e12 * 5.0e-17, rtol=1e-14)


def test_single_absorber_uniform_column_beer_lambert():
    # one absorber of uniform density: tau(k) = sigma n d (N - k - 1/2)
    N, n, d, sig, mu = 6, 1.0e9, 1.0e6, 3.0e-16, 0.5
    J0, s, dl = np.array([2.0e11]), np.array([[7.0e-18]]), np.array([1.5])
    nn = np.zeros((N, 4))
    nn[:, 2] = n
    k = ph.spectral_rates(nn, np.full(N, d), [2], np.array([[sig]]), J0, dl, s, t_f=1.0, mu=mu)
    tau = sig * n * d * (N - np.arange(N) - 0.5)
    np.testing.assert_allclose(k[:, 0], 2.0e11 * 7.0e-18 * 1.5 * np.exp(-tau / mu), rtol=1e-14)


def test_one_bin_reduces_to_the_gray_law():
    # one bin with sigma dlam = 1, t_f = mu = 1: k = J0 exp(-tau), the gray
    # photolysis law of the rate oracle
    rng = np.random.default_rng(3)
    N, S = 8, 5
    n = rng.uniform(1e8, 1e12, (N, S))
    dz = rng.uniform(1e5, 1e6, N)
    sig_tau = 1e-22
    ncol = ph.column_density(n, dz)
    tau = sig_tau * ncol.sum(axis=1)
    k = ph.spectral_rates(n, dz, np.arange(S), np.full((S, 1), sig_tau), np.array([3.0e-4]),
                          np.array([1.0]), np.array([[1.0]]))
    np.testing.assert_allclose(k[:, 0], rates.photolysis(np.log(3.0e-4), tau), rtol=1e-13)


def test_linear_in_tf_and_flux_and_cross_section():
    rng = np.random.default_rng(5)
    N, S, L = 5, 4, 30
    n = rng.uniform(1e8, 1e10, (N, S))
    dz = rng.uniform(1e5, 1e6, N)
    sig_ext = rng.uniform(0, 1e-20, (2, L))
    J0 = rng.uniform(1e10, 1e12, L)
    dl = rng.uniform(0.5, 2, L)
    sig = rng.uniform(0, 1e-18, (3, L))
    k = ph.spectral_rates(n, dz, [1, 3], sig_ext, J0, dl, sig, t_f=0.5, mu=0.7)
    np.testing.assert_allclose(ph.spectral_rates(n, dz, [1, 3], sig_ext, 2 * J0, dl, sig, 0.5, 0.7),
                               2 * k, rtol=1e-14)
    np.testing.assert_allclose(ph.spectral_rates(n, dz, [1, 3], sig_ext, J0, dl, sig, 1.0, 0.7),
                               2 * k, rtol=1e-14)
    k2 = ph.spectral_rates(n, dz, [1, 3], sig_ext, J0, dl, sig[[2, 0]], 0.5, 0.7)
    np.testing.assert_allclose(k2, k[:, [2, 0]], rtol=1e-14)
    # a larger zenith-angle cosine attenuates less
    assert np.all(ph.spectral_rates(n, dz, [1, 3], sig_ext, J0, dl, sig, 0.5, 0.9) >= k)
    # rates grow with height (less column above)
    assert np.all(np.diff(k, axis=0) >= 0)


def test_lagged_spectrum_in_the_step_reduces_to_gray():
    """A one-bin spectrum that reproduces the gray law (sigma dlam = 1, the
    total gas as the single absorber with the gray cross section) gives the
    gray step: the lagged coupling adds nothing else."""
    import synth
    from oracle import integrate
    net = synth.make_network("c2", seed=1002)
    col = synth.make_column("c2", net, seed=301, N=6)
    prob = integrate.Problem(net, col)
    n0 = col.n0
    photo = np.nonzero(np.asarray(net.rtype) == 2)[0]
    lnJ0 = np.asarray(net.params)[photo, 0]
    # one bin per reaction would need per-reaction fluxes: use L = 1 with
    # J0 = 1 and sig_ph = J0_r, and the total gas column as the absorber
    ngas = prob.grid.ngas
    S = n0.shape[1]
    nn = np.concatenate([n0, ngas[:, None]], axis=1)      # extra "species": the total gas
    sp = dict(absorbers=np.array([S]), sig_ext=np.array([[col.sigma_tau]]), J0=np.array([1.0]),
              dlam=np.array([1.0]), sig_ph=np.exp(lnJ0)[:, None], t_f=1.0, mu=1.0)
    kph = __import__("oracle").photolysis.spectral_rates(nn, prob.grid.dz, sp["absorbers"],
                                                         sp["sig_ext"], sp["J0"], sp["dlam"],
                                                         sp["sig_ph"])
    np.testing.assert_allclose(kph, prob.kf[:, photo], rtol=1e-13)
