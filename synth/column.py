"""Seeded synthetic atmospheric columns and batches.

A column is the profile input of the method (Section 2.1 and Fig. P-T
profile): pressure, temperature and eddy-diffusion coefficient per layer
(bottom first), molecular-diffusion coefficients per layer and species,
thermal-diffusion factors, and the initial number densities.  The paper's
HD 189733 b profile (182 layers, from Moses et al. 2011) exists only in a
figure, so log-spaced pressure grids with temperature linear in log P stand
in for it.

Two input-preparation formulas live here because the inputs are specified
through them: the ideal-gas number density used to turn initial mixing
ratios into number densities, and the synthetic molecular-diffusion law
D = 1e21 (T/1000)^0.7 (2/m)^0.5 / n_gas cm^2/s that stands in for the
Chapman-Enskog / binary-mixture coefficients of Section 2.1 (whose
collision data are not available).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .network import make_network

_KB_CGS = 1.380649e-16      # erg/K (exact SI value)
_BAR_CGS = 1.0e6            # dyn/cm^2


@dataclass
class Column:
    P_bar: np.ndarray        # [N] bottom (k=0) to top
    T_K: np.ndarray          # [N]
    Kzz: np.ndarray          # [N] cm^2/s at layer centres
    Dmol: np.ndarray | None  # [N, S] cm^2/s or None (= 0)
    alphaT: np.ndarray | None  # [S] or None (= 0)
    n0: np.ndarray           # [N, S] cm^-3
    mbar_amu: float = 2.3
    g_cgs: float = 2000.0
    sigma_tau: float = 1.0e-22
    seed: int = 0
    info: dict = field(default_factory=dict)
    # boundary fluxes, None = closed: escape at the top (Section 2.4) as 0/1
    # flags for the diffusion-limited velocity and/or set velocities (cm/s),
    # deposition velocities (cm/s) and surface emission fluxes (cm^-2 s^-1)
    # at the bottom (Section 2.5); each [S]
    escape_diff_limited: np.ndarray | None = None
    v_top: np.ndarray | None = None
    v_dep: np.ndarray | None = None
    phi_surf: np.ndarray | None = None

    @property
    def N(self):
        return int(self.P_bar.shape[0])


COLUMN_PRESETS = {
    # 20 layers, 1e2 -> 1e-6 bar, T 2000 -> 1000 K linear in log P,
    # Kzz = 1e8 cm^2/s, no molecular diffusion.
    "c1": dict(N=20, logp=(2.0, -6.0), T=(2000.0, 1000.0), logk=(8.0, 8.0),
               diffusion=False),
    # 120 layers, 1e3 -> 1e-8 bar, T 2500 -> 1000 K, log Kzz 7 -> 10.
    "c2": dict(N=120, logp=(3.0, -8.0), T=(2500.0, 1000.0), logk=(7.0, 10.0),
               diffusion=True),
    # 150 layers, same profile.
    "c3": dict(N=150, logp=(3.0, -8.0), T=(2500.0, 1000.0), logk=(7.0, 10.0),
               diffusion=True),
}


def _number_density(P_bar, T_K):
    return P_bar * _BAR_CGS / (_KB_CGS * T_K)


def synthetic_dmol(P_bar, T_K, mass_amu):
    """Synthetic molecular-diffusion law, [N, S] cm^2/s."""
    ngas = _number_density(P_bar, T_K)
    return (1.0e21 * (T_K[:, None] / 1000.0) ** 0.7
            * np.sqrt(2.0 / mass_amu)[None, :] / ngas[:, None])


def initial_mixing_ratios(net, rng):
    """H2 0.85, He 0.15, others log-uniform in [1e-20, 1e-4] (not renormalised)."""
    S = net.S
    y = 10.0 ** rng.uniform(-20.0, -4.0, S)
    y[0] = 0.85   # H2 is species 0 in every generated network
    y[1] = 0.15   # He is species 1
    return y


def make_column(preset, net, seed, N=None, T_offset=0.0, Kzz_scale=1.0,
                alphaT=None, diffusion=None):
    p = COLUMN_PRESETS[preset]
    N = p["N"] if N is None else int(N)
    rng = np.random.default_rng(seed)
    logp = np.linspace(p["logp"][0], p["logp"][1], N)
    P = 10.0 ** logp
    frac = (logp - p["logp"][0]) / (p["logp"][1] - p["logp"][0])
    T = p["T"][0] + (p["T"][1] - p["T"][0]) * frac + T_offset
    K = 10.0 ** (p["logk"][0] + (p["logk"][1] - p["logk"][0]) * frac) * Kzz_scale
    diff = p["diffusion"] if diffusion is None else diffusion
    D = synthetic_dmol(P, T, net.mass_amu) if diff else None
    y0 = initial_mixing_ratios(net, rng)
    n0 = y0[None, :] * _number_density(P, T)[:, None]
    return Column(P_bar=P, T_K=T, Kzz=K, Dmol=D,
                  alphaT=None if alphaT is None else np.asarray(alphaT, float),
                  n0=np.ascontiguousarray(n0), seed=seed,
                  info=dict(preset=preset, T_offset=T_offset,
                            Kzz_scale=Kzz_scale))


def make_config(c):
    """(network, column) of workload c in {1, 2, 3}; seeds 1000 + c."""
    name = {1: "c1", 2: "c2", 3: "c3"}[c]
    net = make_network(name, seed=1000 + c)
    col = make_column(name, net, seed=1000 + c)
    return net, col


def make_batch(ncols=256, sizes=(90, 250, 594), pool=3, seed=4000,
               n_range=(60, 200)):
    """Ragged batch: column i uses seed 4000 + i.

    Sizes are drawn in equal thirds (seeded); each size has a pool of
    `pool` networks; T offset ~ U[-300, 300] K, Kzz scale ~ log-U[0.1, 10],
    N ~ U{60..200}.
    """
    preset_of = {90: "c2", 250: "s250", 594: "c3"}
    nets = {}
    for s in sizes:
        nets[s] = [make_network(preset_of[s], seed=seed + 100000 + 10 * s + j)
                   for j in range(pool)]
    order = np.random.default_rng(seed).permutation(
        np.repeat(np.arange(len(sizes)), -(-ncols // len(sizes)))[:ncols])
    cols = []
    for i in range(ncols):
        rng = np.random.default_rng(seed + i)
        s = sizes[order[i]]
        net = nets[s][int(rng.integers(0, pool))]
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        dT = float(rng.uniform(-300.0, 300.0))
        ks = float(10.0 ** rng.uniform(-1.0, 1.0))
        col = make_column("c2", net, seed=seed + i, N=N, T_offset=dT,
                          Kzz_scale=ks)
        cols.append((net, col))
    return cols


def make_request(j, net):
    """Serving request j on the 594-species network `net`: the 150-layer
    column of the largest configuration with its own T offset ~ U[-300, 300]
    K, Kzz scale ~ log-U[0.1, 10] and initial abundances (seed 5,000,000 + j)."""
    rng = np.random.default_rng(5_000_000 + j)
    dT = float(rng.uniform(-300.0, 300.0))
    ks = float(10.0 ** rng.uniform(-1.0, 1.0))
    return make_column("c3", net, seed=5_000_000 + j, T_offset=dT, Kzz_scale=ks)


def make_mixed_request(j, nets, n_range=(60, 120)):
    """Serving request j of the two-size stream: network nets[size] with
    the size drawn from the keys of nets (equal odds), the 120-layer
    profile's pressure range on N ~ U{n_range} layers, T offset ~ U[-300,
    300] K, Kzz scale ~ log-U[0.1, 10] and its own initial abundances
    (seed 6,000,000 + j).  Returns (size, column)."""
    rng = np.random.default_rng(6_000_000 + j)
    sizes = sorted(nets)
    size = sizes[int(rng.integers(0, len(sizes)))]
    N = int(rng.integers(n_range[0], n_range[1] + 1))
    dT = float(rng.uniform(-300.0, 300.0))
    ks = float(10.0 ** rng.uniform(-1.0, 1.0))
    return size, make_column("c2", nets[size], seed=6_000_000 + j, N=N, T_offset=dT,
                             Kzz_scale=ks)


def poisson_arrivals(n, rate, seed=5_000_000):
    """Arrival times (s) of n requests at a Poisson rate (per second)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def make_spectrum(net, L=10000, seed=7000):
    """Wavelength grid, top-of-atmosphere flux and cross sections for the
    spectral photolysis rates of net's photolysis reactions (Section 2.3.3:
    10,000 bins of about 1 A from 1 to 10,000 A).  Returns a dict:
      lam, dlam [L] (A); J0 [L] photons cm^-2 s^-1 A^-1 (a smooth stellar-like
      shape falling into the far UV); photo [P] reaction indices; sig_ph [P, L]
      cm^2, one Gaussian band per reaction (centre 900-3000 A, width 30-300 A,
      peak 1e-19 to 1e-17 cm^2) cut off beyond 4 widths; absorbers [A] the
      distinct photolysed species; sig_ext [A, L] cm^2, the sum of their
      reactions' bands plus a Rayleigh-like 1e-27 (5000/lam)^4 term.
    Inputs only: no rate, flux attenuation or optical depth is evaluated."""
    rng = np.random.default_rng(seed)
    lam = np.linspace(1.0, 10000.0, L) if L > 1 else np.array([2000.0])
    dlam = np.full(L, (lam[-1] - lam[0]) / max(L - 1, 1) if L > 1 else 1.0)
    x = lam / 5000.0
    J0 = 1e13 * x ** 3 / np.expm1(np.minimum(2.5 / x, 50.0))
    photo = np.nonzero(np.asarray(net.rtype) == 2)[0]
    P = len(photo)
    sig_ph = np.zeros((P, L))
    centre = rng.uniform(900.0, 3000.0, P)
    width = rng.uniform(30.0, 300.0, P)
    peak = 10.0 ** rng.uniform(-19.0, -17.0, P)
    for p in range(P):
        u = (lam - centre[p]) / width[p]
        band = peak[p] * np.exp(-0.5 * u * u)
        band[np.abs(u) > 4.0] = 0.0
        sig_ph[p] = band
    reac = np.asarray(net.reac)[photo, 0] if P else np.zeros(0, int)
    absorbers = np.unique(reac).astype(np.int32)
    sig_ext = np.zeros((len(absorbers), L))
    for a, sp in enumerate(absorbers):
        sig_ext[a] = sig_ph[reac == sp].sum(axis=0) + 1e-27 * (5000.0 / lam) ** 4
    return dict(lam=lam, dlam=dlam, J0=J0, photo=photo.astype(np.int32), sig_ph=sig_ph,
                absorbers=absorbers, sig_ext=sig_ext)


def with_boundary(net, col, seed=8000, open_top=True, open_bottom=True):
    """A copy of col with boundary exchange (Sections 2.4, 2.5): the species
    lighter than the mean molecular mass flagged for diffusion-limited escape
    (the paper's H/He case), set escape velocities of 0.1-10 cm/s on 10 % of
    the others (its user-defined case), deposition velocities of 1e-3-1 cm/s
    on 30 % of the species and surface emission of 1e8-1e11 cm^-2 s^-1 on
    10 %, log-uniform, and at least one species of each kind.  Inputs only:
    no velocity or flux is derived here."""
    import dataclasses
    rng = np.random.default_rng(seed)
    S = len(net.mass_amu)
    light = (np.asarray(net.mass_amu) < col.mbar_amu).astype(np.int32)
    pick_top = (rng.random(S) < 0.1) & (light == 0)
    v_top = np.where(pick_top, 10.0 ** rng.uniform(-1.0, 1.0, S), 0.0)
    v_dep = np.where(rng.random(S) < 0.3, 10.0 ** rng.uniform(-3.0, 0.0, S), 0.0)
    phi = np.where(rng.random(S) < 0.1, 10.0 ** rng.uniform(8.0, 11.0, S), 0.0)
    # at least one species of each kind, also on small networks
    for arr, lo, hi, allowed in ((v_top, -1.0, 1.0, light == 0), (v_dep, -3.0, 0.0, None),
                                 (phi, 8.0, 11.0, None)):
        if not (arr > 0).any():
            idx = np.nonzero(allowed)[0] if allowed is not None else np.arange(S)
            if len(idx):
                arr[rng.choice(idx)] = 10.0 ** rng.uniform(lo, hi)
    return dataclasses.replace(
        col,
        escape_diff_limited=light if open_top else None,
        v_top=v_top if open_top else None,
        v_dep=v_dep if open_bottom else None,
        phi_surf=phi if open_bottom else None)
