"""Seeded synthetic reaction networks.

What is drawn, and why (the paper's networks are available only on request,
Data Availability section, so these stand in for them at their sizes):

* Species are element compositions over C/H/O/N (+P, S and six metals for
  the 594-species instances, like the C-H-O-N-P-S-Metals network of
  Section 2.2).  H2 and He are always present; He is inert.  Compositions
  are drawn by "sum closure" (a new species is often the sum of two
  existing ones) so that element-balanced reactions are plentiful.
* Reactions come in the three families of Section 2.3: two-body
  A+B->C+D, three-body recombinations A+B(+M)->C and photolysis A->B+C.
  Every reaction is element-balanced by construction (equal atom totals
  on both sides), which is what makes element conservation a test.
* Rate-law parameters are drawn from the ranges of the workload
  (log10 A ~ U[-16,-9] cm^3/s, b ~ U[-2,2], C ~ U[0,30000] K for the
  two-body law; low-pressure limits log10 A0 ~ U[-34,-28] cm^6/s,
  b0 ~ U[-2,0], C0 ~ U[0,5000] K; J0 ~ log-U[1e-8,1e-3] 1/s) and redrawn
  while the parameters fall outside an acceptance region that keeps every
  two-body coefficient below the collisional limit (Section 2.2 excludes
  such reactions).  The region is a bound on the parameters themselves:
  log10 A + max(b log10 Tb_lo, b log10 Tb_hi) <= LOG10_PREFAC_MAX, which
  bounds A*Tb^b and hence the rate, since exp(-C/T) <= 1 for C >= 0.
* Thermochemistry is a single-range NASA-7 set per species (a2..a5 = 0,
  identical low and high ranges) built from per-element contributions plus
  a bond term and a small per-species perturbation.  For an element-balanced
  two-body reaction the element and bond parts cancel, so the reverse
  coefficient differs from the forward one only through the perturbations;
  each two-body reaction is oriented so that its a6 sum does not increase
  (exothermic forward), which keeps the reverse coefficient within a factor
  of about 10^2.1 of the forward one.  Three-body recombinations release one
  bond energy, so their reverse (thermal decomposition) is slow when cool
  and fast when hot.

Nothing in this file evaluates a rate coefficient or a Gibbs energy.
"""

from __future__ import annotations

import collections
from dataclasses import dataclass, field

import numpy as np

# Standard atomic weights (amu).  The six "metals" are real metals used as
# synthetic elements for the 594-species networks.
ATOMIC_MASS = {
    "H": 1.008, "He": 4.002602, "C": 12.011, "N": 14.007, "O": 15.999,
    "P": 30.973762, "S": 32.06, "Na": 22.98976928, "Mg": 24.305,
    "Al": 26.9815385, "K": 39.0983, "Ca": 40.078, "Fe": 55.845,
}

CHON = ["H", "He", "C", "O", "N"]
CHONPS_METALS = ["H", "He", "C", "O", "N", "P", "S", "Na", "Mg", "Al", "K",
                 "Ca", "Fe"]

MAX_REAC = 3
MAX_PROD = 3
RT_BIMOL, RT_TERMOL, RT_PHOTO = 0, 1, 2

# Two-body coefficients must stay under 1e-8 cm^3/s (collisional limit).  The
# forward prefactor bound leaves 10^2.1 of room for the reverse coefficient:
# for an exothermic-forward two-body reaction the reverse/forward ratio is
# at most exp(|d1| max|1 - ln T| + |d7|) <= exp(0.4*7 + 2) < 10^2.1 with the
# perturbation ranges below (T < 2980 K).
LOG10_PREFAC_MAX = -10.1


@dataclass
class Network:
    """Plain arrays describing one reaction network (host memory)."""
    elements: list
    species: list            # formula strings, for reports only
    elem_comp: np.ndarray    # int32 [E, S] atom counts
    mass_amu: np.ndarray     # float64 [S]
    nasa7: np.ndarray        # float64 [S, 2, 7]; [:,0] low range, [:,1] high
    t_mid: float             # high range used iff T >= t_mid
    rtype: np.ndarray        # int32 [R]
    reac: np.ndarray         # int32 [R, MAX_REAC], -1 padded
    prod: np.ndarray         # int32 [R, MAX_PROD], -1 padded
    reversible: np.ndarray   # int32 [R]
    tb_kooij: np.ndarray     # int32 [R]; 1: T_b = T/300, 0: T_b = T
    params: np.ndarray       # float64 [R, 6]
    t_range: tuple = (1000.0, 2000.0)
    seed: int = 0
    info: dict = field(default_factory=dict)

    @property
    def S(self):
        return int(self.elem_comp.shape[1])

    @property
    def R(self):
        return int(self.rtype.shape[0])

    @property
    def E(self):
        return int(self.elem_comp.shape[0])


# name -> (S, elements, n_bimol, n_termol, n_photo, T range, kooij fraction,
#          max atoms per species, sum-closure probability, element weights)
NETWORK_PRESETS = {
    # 12 species / 30 two-body reactions over C/H/O/N, modified Arrhenius only.
    "c1": dict(S=12, elements=CHON, n_bi=30, n_ter=0, n_ph=0,
               t_range=(1000.0, 2000.0), kooij_frac=0.0, max_atoms=4,
               p_sum=0.6, weights={"H": .4, "C": .3, "O": .2, "N": .1}),
    # 12 species with two-body and three-body reactions and no photolysis:
    # small closed-layer equilibrium checks.
    "t12": dict(S=12, elements=CHON, n_bi=20, n_ter=8, n_ph=0,
                t_range=(700.0, 2800.0), kooij_frac=0.3, max_atoms=4,
                p_sum=0.6, weights={"H": .4, "C": .3, "O": .2, "N": .1}),
    # 48 species / 500 reactions (padded block size 64), same mix as c2.
    "s48": dict(S=48, elements=CHON, n_bi=400, n_ter=50, n_ph=50,
                t_range=(700.0, 2800.0), kooij_frac=0.3, max_atoms=5,
                p_sum=0.5, weights=None),
    # 90 species / 1200 reactions, 80/10/10 two-body/three-body/photolysis.
    "c2": dict(S=90, elements=CHON, n_bi=960, n_ter=120, n_ph=120,
               t_range=(700.0, 2800.0), kooij_frac=0.3, max_atoms=6,
               p_sum=0.5, weights=None),
    # 250 species, same reactions-per-species ratio (batched mix).
    "s250": dict(S=250, elements=CHONPS_METALS, n_bi=2600, n_ter=325,
                 n_ph=325, t_range=(700.0, 2800.0), kooij_frac=0.3,
                 max_atoms=6, p_sum=0.5, weights=None),
    # 594 species / 7720 reactions (the size of XODIAC-2025, Section 2.2).
    "c3": dict(S=594, elements=CHONPS_METALS, n_bi=6176, n_ter=772, n_ph=772,
               t_range=(700.0, 2800.0), kooij_frac=0.3, max_atoms=6,
               p_sum=0.5, weights=None),
}


def _formula(comp, elements):
    parts = []
    for e, n in zip(elements, comp):
        if n:
            parts.append(e + (str(n) if n > 1 else ""))
    return "".join(parts)


def _draw_compositions(S, elements, rng, max_atoms, p_sum, weights):
    E = len(elements)
    iH, iHe = elements.index("H"), elements.index("He")
    reactive = [e for e in range(E) if e != iHe]
    if weights is None:
        w = np.ones(len(reactive))
        w[reactive.index(iH)] = 3.0
    else:
        w = np.array([weights.get(elements[e], 0.0) for e in reactive])
    w = w / w.sum()
    h2 = tuple(2 if e == iH else 0 for e in range(E))
    he = tuple(1 if e == iHe else 0 for e in range(E))
    comps = [h2, he]
    seen = set(comps)
    tries = 0
    while len(comps) < S:
        tries += 1
        if tries > 200000:
            raise RuntimeError("composition draw did not fill the species list")
        if len(comps) > 3 and rng.random() < p_sum:
            i, j = rng.integers(0, len(comps), 2)
            if comps[i][iHe] or comps[j][iHe]:
                continue
            c = tuple(int(a + b) for a, b in zip(comps[i], comps[j]))
            if sum(c) > max_atoms:
                continue
        else:
            nat = int(rng.integers(1, 3))
            c = [0] * E
            for _ in range(nat):
                c[reactive[rng.choice(len(reactive), p=w)]] += 1
            c = tuple(c)
        if c in seen:
            continue
        seen.add(c)
        comps.append(c)
    return np.array(comps, dtype=np.int64)


def _candidates(comp, iHe):
    """Balanced candidate reactions, in a deterministic order.

    Returns (bimol, triples): bimol is a list of ((A,B),(C,D)) with equal
    composition sums; triples is a list of (A,B,C) with comp A + comp B =
    comp C.  He (inert) takes part in none.
    """
    S = comp.shape[0]
    index = {tuple(c): i for i, c in enumerate(comp)}
    sums = collections.OrderedDict()
    for i in range(S):
        if comp[i, iHe]:
            continue
        for j in range(i, S):
            if comp[j, iHe]:
                continue
            sums.setdefault(tuple(comp[i] + comp[j]), []).append((i, j))
    bimol, triples = [], []
    for key, pairs in sums.items():
        for p in range(len(pairs)):
            for q in range(p + 1, len(pairs)):
                bimol.append((pairs[p], pairs[q]))
        c = index.get(key)
        if c is not None:
            for (i, j) in pairs:
                triples.append((i, j, c))
    return bimol, triples


def _draw_thermo(comp, elements, rng):
    """Single-range NASA-7 coefficients: element parts + bond term + noise."""
    E = len(elements)
    S = comp.shape[0]
    c_e = rng.uniform(0.8, 1.6, E)        # a1 per atom
    h_e = rng.uniform(-2.0e4, 2.0e4, E)   # a6 per atom [K]
    s_e = rng.uniform(-1.0, 3.0, E)       # a7 per atom
    bond = rng.uniform(3.0e4, 4.0e4)      # a6 released per bond formed [K]
    d1 = rng.uniform(-0.1, 0.1, S)
    d6 = rng.uniform(-4000.0, 4000.0, S)
    d7 = rng.uniform(-0.5, 0.5, S)
    natoms = comp.sum(axis=1)
    a1 = 1.5 + comp @ c_e + d1
    a6 = comp @ h_e - bond * (natoms - 1) + d6
    a7 = comp @ s_e + d7
    nasa = np.zeros((S, 2, 7))
    for r in range(2):
        nasa[:, r, 0] = a1
        nasa[:, r, 5] = a6
        nasa[:, r, 6] = a7
    return nasa, dict(bond=float(bond))


def _draw_arrhenius(rng, t_lo, t_hi, kooij, la_rng=(-16.0, -9.0),
                    b_rng=(-2.0, 2.0), c_rng=(0.0, 30000.0),
                    log10_max=LOG10_PREFAC_MAX):
    """(ln A, b, C) drawn from the workload ranges inside the acceptance region."""
    lo, hi = (t_lo / 300.0, t_hi / 300.0) if kooij else (t_lo, t_hi)
    llo, lhi = np.log10(lo), np.log10(hi)
    for _ in range(100000):
        la = rng.uniform(*la_rng)
        b = rng.uniform(*b_rng)
        if la + max(b * llo, b * lhi) <= log10_max:
            c = rng.uniform(*c_rng)
            return la * np.log(10.0), b, c
    raise RuntimeError("acceptance region too small")


def make_network(preset="c1", seed=1001, max_retries=5000):
    """Draw one network of a preset shape (see NETWORK_PRESETS)."""
    p = NETWORK_PRESETS[preset]
    S, elements = p["S"], list(p["elements"])
    n_bi, n_ter, n_ph = p["n_bi"], p["n_ter"], p["n_ph"]
    t_lo, t_hi = p["t_range"]
    rng = np.random.default_rng(seed)
    iHe = elements.index("He")
    for attempt in range(max_retries):
        comp = _draw_compositions(S, elements, rng, p["max_atoms"], p["p_sum"],
                                  p["weights"])
        bimol, triples = _candidates(comp, iHe)
        if len(bimol) >= n_bi and len(triples) >= max(n_ter, n_ph):
            break
    else:
        raise RuntimeError(f"no composition set with enough reactions ({preset})")

    nasa, thermo_info = _draw_thermo(comp, elements, rng)
    a6 = nasa[:, 0, 5]

    R = n_bi + n_ter + n_ph
    rtype = np.zeros(R, np.int32)
    reac = -np.ones((R, MAX_REAC), np.int32)
    prod = -np.ones((R, MAX_PROD), np.int32)
    reversible = np.zeros(R, np.int32)
    tb_kooij = np.zeros(R, np.int32)
    params = np.zeros((R, 6))

    r = 0
    sel = rng.permutation(len(bimol))[:n_bi]
    for s in sorted(sel):
        (A, B), (C, D) = bimol[s]
        # Orient exothermic-forward: the a6 sum must not increase.
        if a6[C] + a6[D] > a6[A] + a6[B]:
            (A, B), (C, D) = (C, D), (A, B)
        kooij = rng.random() < p["kooij_frac"]
        la, b, c = _draw_arrhenius(rng, t_lo, t_hi, kooij)
        rtype[r] = RT_BIMOL
        reac[r, :2] = (A, B)
        prod[r, :2] = (C, D)
        reversible[r] = 1
        tb_kooij[r] = int(kooij)
        params[r, :3] = (la, b, c)
        r += 1
    if n_ter:
        sel = rng.permutation(len(triples))[:n_ter]
        for s in sorted(sel):
            A, B, C = triples[s]
            kooij = rng.random() < p["kooij_frac"]
            la0, b0, c0 = _draw_arrhenius(rng, t_lo, t_hi, kooij,
                                          la_rng=(-34.0, -28.0),
                                          b_rng=(-2.0, 0.0),
                                          c_rng=(0.0, 5000.0),
                                          log10_max=np.inf)
            lai, bi, ci = _draw_arrhenius(rng, t_lo, t_hi, kooij)
            rtype[r] = RT_TERMOL
            reac[r, :2] = (A, B)
            prod[r, 0] = C
            reversible[r] = 1
            tb_kooij[r] = int(kooij)
            params[r] = (la0, b0, c0, lai, bi, ci)
            r += 1
    if n_ph:
        sel = rng.permutation(len(triples))[:n_ph]
        for s in sorted(sel):
            A, B, C = triples[s]
            rtype[r] = RT_PHOTO
            reac[r, 0] = C
            prod[r, :2] = (A, B)
            reversible[r] = 0
            params[r, 0] = rng.uniform(-8.0, -3.0) * np.log(10.0)  # ln J0
            r += 1
    assert r == R

    species = [_formula(c, elements) for c in comp]
    mass = comp @ np.array([ATOMIC_MASS[e] for e in elements])
    return Network(
        elements=elements, species=species,
        elem_comp=np.ascontiguousarray(comp.T.astype(np.int32)),
        mass_amu=mass.astype(np.float64), nasa7=nasa, t_mid=1000.0,
        rtype=rtype, reac=reac, prod=prod, reversible=reversible,
        tb_kooij=tb_kooij, params=params, t_range=(t_lo, t_hi), seed=seed,
        info=dict(preset=preset, composition_attempts=attempt + 1,
                  n_bimol_candidates=len(bimol),
                  n_triple_candidates=len(triples), **thermo_info))


def small_network(species_comp, elements, reactions, nasa7, mass_amu=None):
    """Hand-built network for closed-form tests.

    reactions: list of dicts with keys type ('bi'|'ter'|'ph'), reac, prod,
    params (len <= 6), reversible (bool), kooij (bool).
    """
    comp = np.asarray(species_comp, dtype=np.int32)  # [S, E]
    S = comp.shape[0]
    R = len(reactions)
    rtype = np.zeros(R, np.int32)
    reac = -np.ones((R, MAX_REAC), np.int32)
    prod = -np.ones((R, MAX_PROD), np.int32)
    rev = np.zeros(R, np.int32)
    kooij = np.zeros(R, np.int32)
    params = np.zeros((R, 6))
    code = {"bi": RT_BIMOL, "ter": RT_TERMOL, "ph": RT_PHOTO}
    for i, rx in enumerate(reactions):
        rtype[i] = code[rx["type"]]
        reac[i, :len(rx["reac"])] = rx["reac"]
        prod[i, :len(rx["prod"])] = rx["prod"]
        rev[i] = int(rx.get("reversible", rx["type"] != "ph"))
        kooij[i] = int(rx.get("kooij", False))
        params[i, :len(rx["params"])] = rx["params"]
    if mass_amu is None:
        mass_amu = comp @ np.array([ATOMIC_MASS.get(e, 1.0) for e in elements])
    species = [_formula(c, elements) for c in comp]
    return Network(elements=list(elements), species=species,
                   elem_comp=np.ascontiguousarray(comp.T),
                   mass_amu=np.asarray(mass_amu, np.float64),
                   nasa7=np.asarray(nasa7, np.float64).reshape(S, 2, 7),
                   t_mid=1000.0, rtype=rtype, reac=reac, prod=prod,
                   reversible=rev, tb_kooij=kooij, params=params,
                   t_range=(100.0, 3000.0), seed=0, info={})
