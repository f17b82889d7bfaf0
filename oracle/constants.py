"""Units of the oracle: Angstrom, fs, amu, eV (CODATA 2018 values)."""
KB = 8.617333262e-5                 # Boltzmann constant, eV/K
HBAR = 0.6582119569                 # reduced Planck constant, eV fs
# 1 amu A^2 / fs^2 in eV: 1.66053906660e-27 kg * 1e-20 m^2 / 1e-30 s^2 / 1.602176634e-19 J
MVV2E = 1.66053906660e-27 * 1e10 / 1.602176634e-19
