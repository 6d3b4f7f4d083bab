"""Spectral photolysis rate coefficients (Section 2.3.3).  Test
infrastructure only: the HIP library never imports this module.

Definitions followed, with the readings taken:
  * actinic flux (Eq. of the total actinic flux): J(z, lam) = J0(lam)
    exp(-tau(z, lam)/mu) + J_diff, with J_diff = 0 (no diffuse component,
    as in the gray treatment of the rates);
  * optical depth (Eq. of the total extinction): tau = sum_i (sigma_a,i +
    sigma_s,i) n_i dz, summed over the absorbing species i and over the
    layers above the point: at the midpoint of layer k the column of
    species i is N_i(k) = n_i,k dz_k / 2 + sum_{j>k} n_i,j dz_j (the same
    half-layer reading as the gray optical depth of the column grid);
    sigma_ext,i = sigma_a,i + sigma_s,i is one input table per absorber;
  * rate coefficient (Eq. of k_ph): k_ph,r(z) = t_f int J(z, lam)
    sigma_r(lam) dlam, the integral taken as the sum over wavelength bins
    b of J(z, lam_b) sigma_r(lam_b) dlam_b.
parity: pinned by closed forms (optically thin box bands, a single absorber
in a uniform column), by the gray law of oracle.rates.photolysis for one
bin, and by the linearity and scaling invariants (tests).
"""

import numpy as np


def column_density(n_abs, dz):
    """N[k, a] = n[k, a] dz[k] / 2 + sum_{j > k} n[j, a] dz[j] (layer 0 at the
    bottom), by one pass from the top layer down."""
    n_abs = np.asarray(n_abs, float)
    N = n_abs.shape[0]
    out = np.zeros_like(n_abs)
    above = np.zeros(n_abs.shape[1])
    for k in range(N - 1, -1, -1):
        out[k] = above + 0.5 * n_abs[k] * dz[k]
        above = above + n_abs[k] * dz[k]
    return out


def optical_depth(ncol, sig_ext):
    """tau[k, b] = sum_a ncol[k, a] sig_ext[a, b]."""
    return np.asarray(ncol, float) @ np.asarray(sig_ext, float)


def actinic_flux(J0, tau, mu):
    """J[k, b] = J0[b] exp(-tau[k, b] / mu) (no diffuse component)."""
    return np.asarray(J0, float)[None, :] * np.exp(-np.asarray(tau, float) / mu)


def spectral_rates(n, dz, absorbers, sig_ext, J0, dlam, sig_ph, t_f=1.0, mu=1.0):
    """k_ph[k, p] = t_f sum_b J(k, lam_b) sig_ph[p, b] dlam[b].

    n [N, S] number densities, dz [N] layer thicknesses, absorbers [A]
    species indices with extinction cross sections sig_ext [A, L], J0 [L]
    top-of-atmosphere flux per unit wavelength, dlam [L] bin widths,
    sig_ph [P, L] photodissociation cross sections of the P reactions."""
    n = np.asarray(n, float)
    ncol = column_density(n[:, np.asarray(absorbers, int)], np.asarray(dz, float))
    tau = optical_depth(ncol, sig_ext)
    J = actinic_flux(J0, tau, mu)
    return t_f * (J * np.asarray(dlam, float)[None, :]) @ np.asarray(sig_ph, float).T
