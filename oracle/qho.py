"""Quantum harmonic oscillator closed forms (oracle side, Sec. S1).

One Cartesian degree of freedom of mass m (amu) and angular frequency w
(1/fs) at temperature T; spring constant k = m w^2 MVV2E (eV/A^2).

Exact quantum:   <x^2> = hbar / (2 m w MVV2E) coth(beta hbar w / 2),
                 <E>   = hbar w / 2 coth(beta hbar w / 2);
classical:       <x^2> = 1 / (beta k),  <E> = k_B T.
P beads (the ring polymer of Sec. 2.1 with its normal modes): mode l has
stiffness k + m w_l^2 MVV2E with w_l = 2 w_P sin(l pi / P), w_P = P/(beta hbar),
and every bead carries the mean of the mode variances:
  <x^2>_P = 1/(beta k) sum_{l=0}^{P-1} [1 + (2P/(beta hbar w))^2 sin^2(l pi/P)]^-1.
(The bead sum printed in Sec. S1 lacks this square and mixes a factor 3k_BT
from three dimensions into the one-dimensional case; the sum above is the
finite-P result it stands for.)  The virial energy estimator gives
<E>_P = k <x^2>_P, because <K> = <V> for the harmonic well.
Closed form of the sum:
  <x^2>_P = hbar/(2 m w MVV2E) coth(P asinh(a)) / sqrt(1 + a^2),  a = beta hbar w / (2P).
"""
import numpy as np

from .constants import KB, HBAR, MVV2E


def x2_exact(m, w, T):
    beta = 1.0 / (KB * T)
    return HBAR / (2.0 * m * w * MVV2E) / np.tanh(beta * HBAR * w / 2.0)


def energy_exact(w, T):
    beta = 1.0 / (KB * T)
    return 0.5 * HBAR * w / np.tanh(beta * HBAR * w / 2.0)


def x2_classical(m, w, T):
    return KB * T / (m * w * w * MVV2E)


def x2_beads_sum(m, w, T, P):
    beta = 1.0 / (KB * T)
    l = np.arange(P)
    return x2_classical(m, w, T) * np.sum(1.0 / (1.0 + (2.0 * P / (beta * HBAR * w)) ** 2
                                                 * np.sin(l * np.pi / P) ** 2))


def x2_beads_closed(m, w, T, P):
    beta = 1.0 / (KB * T)
    a = beta * HBAR * w / (2.0 * P)
    return HBAR / (2.0 * m * w * MVV2E) / np.tanh(P * np.arcsinh(a)) / np.sqrt(1.0 + a * a)


def energy_beads(m, w, T, P):
    return m * w * w * MVV2E * x2_beads_sum(m, w, T, P)
