"""Element-potential chemical equilibrium at fixed T and volume.
Test infrastructure only.

Independent of the kinetic path: with every reaction reversible through
K_c = exp(-Delta g)(P0/(k_B T))^Delta nu (Section 2.3.4), the kinetic steady
state of a closed layer satisfies detailed balance, i.e.
ln(n_y / n_ref) + g_y = sum_e lambda_e a_{e,y} with n_ref = P0/(k_B T).
Given element totals b_e, the potentials lambda solve
sum_y a_{e,y} n_y(lambda) = b_e, the stationarity condition of the convex
function phi(lambda) = sum_y n_y(lambda) - sum_e lambda_e b_e.  Newton's
method with backtracking on phi finds them.
"""

import numpy as np

from .constants import KB, P_STD
from .thermo import species_g


def equilibrium_layer(nasa7, t_mid, elem_comp, T, b, lam0=None, tol=1e-12,
                      max_iter=2000):
    """Number densities [S] at equilibrium for element totals b [E]."""
    A = np.asarray(elem_comp, float)          # [E, S]
    g = species_g(nasa7, t_mid, T)
    ln_ref = np.log(P_STD / (KB * T))
    E = A.shape[0]
    lam = np.zeros(E) if lam0 is None else np.array(lam0, float)

    def dens(l):
        return np.exp(ln_ref - g + A.T @ l)

    def phi(l):
        return dens(l).sum() - l @ b

    for _ in range(max_iter):
        n = dens(lam)
        r = A @ n - b
        if np.all(np.abs(r) <= tol * b):
            return n, lam
        H = (A * n) @ A.T
        step = np.linalg.solve(H, -r)
        big = np.max(np.abs(step))
        if big < 1e-13:        # converged to rounding
            return dens(lam + step), lam + step
        if big > 5.0:          # keep trial densities within exp(5 * max atoms)
            step *= 5.0 / big
        f0, s = phi(lam), 1.0
        # Near the solution phi is flat to rounding: take full Newton steps.
        if big > 0.1:
            while phi(lam + s * step) > f0 - 1e-4 * s * (r @ -step) and s > 1e-12:
                s *= 0.5
        lam = lam + s * step
    raise RuntimeError("element-potential Newton did not converge")


def initial_potentials(nasa7, t_mid, elem_comp, T, n):
    """Least-squares fit of ln(n/n_ref) + g = A^T lambda: a starting point."""
    A = np.asarray(elem_comp, float)
    g = species_g(nasa7, t_mid, T)
    mu = np.log(np.maximum(n, 1e-300) / (P_STD / (KB * T))) + g
    lam, *_ = np.linalg.lstsq(A.T, mu, rcond=None)
    return lam
