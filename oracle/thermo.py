"""NASA 7-coefficient thermochemistry (Appendix A, G/RT and Cp/R polynomials).

Test infrastructure only.
"""

import numpy as np


def g_over_rt(a, T):
    """Dimensionless standard Gibbs energy G/RT of one coefficient set.

    Appendix A: G/RT = a1 (1 - ln T) - a2 T/2 - a3 T^2/6 - a4 T^3/12
                       - a5 T^4/20 + a6/T - a7.
    """
    a1, a2, a3, a4, a5, a6, a7 = (float(x) for x in a)
    return (a1 * (1.0 - np.log(T)) - a2 * T / 2.0 - a3 * T ** 2 / 6.0
            - a4 * T ** 3 / 12.0 - a5 * T ** 4 / 20.0 + a6 / T - a7)


def cp_over_r(a, T):
    """Appendix A: Cp/R = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4."""
    a1, a2, a3, a4, a5 = (float(x) for x in a[:5])
    return a1 + a2 * T + a3 * T ** 2 + a4 * T ** 3 + a5 * T ** 4


def species_g(nasa7, t_mid, T):
    """G/RT of every species at temperature T; the high range is used iff
    T >= t_mid (Appendix A gives 10-1000 K and 1000-3000 K ranges; the tie
    at exactly t_mid goes to the high range)."""
    rng = 1 if T >= t_mid else 0
    return np.array([g_over_rt(nasa7[y, rng], T) for y in range(nasa7.shape[0])])
