"""Physical constants in CGS (oracle side; test infrastructure only)."""

KB = 1.380649e-16          # Boltzmann constant, erg/K (exact SI definition)
AMU = 1.66053906660e-24    # atomic mass unit, g (CODATA 2018)
P_STD = 1.0e6              # standard pressure 1 bar in dyn/cm^2
