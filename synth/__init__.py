"""Seeded synthetic inputs for the implicit photochemical column solver.

This package draws the *inputs* that both the CPU oracle and the HIP library
consume: chemical networks (species compositions, reactions, rate-law
parameters, NASA-7 thermochemical coefficients) and atmospheric columns
(pressure, temperature and eddy-diffusion profiles, molecular-diffusion
coefficients, initial number densities).  It contains no part of the
method's arithmetic: no rate coefficient, Gibbs energy, flux, Jacobian or
solve is ever evaluated here.  The recipes stand in for the paper's
networks (STAND-2020, SNCHO, XODIAC-2025; Section 2.2) and the
HD 189733 b profile (Section 3, Fig. P-T profile), which are not public,
at their shapes and sizes.
"""

from .network import make_network, NETWORK_PRESETS
from .column import (make_column, COLUMN_PRESETS, make_config, make_batch, make_request,
                     make_mixed_request, poisson_arrivals, make_spectrum, with_boundary)

__all__ = ["make_network", "make_column", "make_config", "make_batch", "make_request",
           "make_mixed_request",
           "poisson_arrivals", "make_spectrum", "with_boundary",
           "NETWORK_PRESETS", "COLUMN_PRESETS"]
