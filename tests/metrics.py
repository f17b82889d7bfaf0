"""Error metrics of the parity tests.

force error   e_i = |F_i - F_i^ref| / max(|F_i^ref|, 0.1 F_rms^ref), reported as max_i e_i;
bead energy   |E_b - E_b^ref| / sum_i |E_i^ref| (sum over the atoms of the bead),
so cancellation in random-weight energies does not inflate the error.
"""
import numpy as np


def force_error(F, F_ref):
    F = np.asarray(F, dtype=np.float64).reshape(-1, 3)
    F_ref = np.asarray(F_ref, dtype=np.float64).reshape(-1, 3)
    nref = np.linalg.norm(F_ref, axis=1)
    floor = 0.1 * np.sqrt(np.mean(nref ** 2))
    return float(np.max(np.linalg.norm(F - F_ref, axis=1) / np.maximum(nref, floor)))


def energy_error(E, E_ref, abs_atom_sum):
    E = np.asarray(E, dtype=np.float64)
    return float(np.max(np.abs(E - E_ref) / np.asarray(abs_atom_sum)))


def rel_max(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(a - ref)) / max(np.max(np.abs(ref)), 1e-300))
