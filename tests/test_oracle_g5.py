"""Pins of the oracle's G5 angular functions (the angular sum without the
factors that involve r_jk) and of the forces of a network built on them.

The expectations come from outside the oracle's double loop over neighbour
pairs: closed forms for two neighbours, the spherical-harmonic addition
theorem (scipy's harmonics and numpy's Legendre conversion) applied to
random clusters, the G4 functions in the limit where the r_jk factors are 1,
and central finite differences of the FP64 energy.
"""
import dataclasses
import math

import numpy as np
import pytest
from numpy.polynomial import legendre
from scipy import special

from oracle import bpnn, neighbors
from paper_2503_23728_amd import synthetic as S

RC = 6.0


def _model(angular="g5", elements=("H", "O"), n_ang=16, seed=5):
    m = S.make_model(list(elements), 16, n_ang, [32, 16], seed)
    return dataclasses.replace(m, angular=angular)


def _fc(r, rc=RC):
    return 0.5 * (math.cos(math.pi * r / rc) + 1.0) if r < rc else 0.0


def _G(model, q, species, box=np.zeros(3)):
    q = np.asarray(q, dtype=np.float64)
    start, idx = neighbors.brute_force_fp32(q.astype(np.float32), box, model.cutoff)
    return bpnn.descriptors(model, q, np.asarray(species, np.int32), box, np.arange(len(q)), start, idx)


def _ang_index(model, e1, e2, ieta, zeta, lam):
    n_el = model.n_elements
    a, b = min(e1, e2), max(e1, e2)
    pair = a * n_el - a * (a - 1) // 2 + (b - a)
    return n_el * model.n_rad + pair * model.n_ang + (ieta * 4 + S.ZETAS.index(zeta)) * 2 + (0 if lam > 0 else 1)


def test_two_neighbours_right_angle_closed_form():
    m = _model()
    b, c = 1.5, 2.5
    G = _G(m, [[0, 0, 0], [b, 0, 0], [0, c, 0]], [0, 1, 0])
    for ie, eta in enumerate(m.ang_eta):
        for zeta in S.ZETAS:
            for lam in S.LAMBDAS:
                want = 2.0 ** (1 - zeta) * math.exp(-eta * (b * b + c * c)) * _fc(b) * _fc(c)
                assert G[0, _ang_index(m, 0, 1, ie, zeta, lam)] == pytest.approx(want, rel=1e-12)


def test_far_pair_counts_in_g5_only():
    # j and k on opposite sides of i, 10 A apart (> R_c): cos = -1; G4 drops the
    # pair (f_c(r_jk) = 0), G5 keeps it: (1 - lambda)^zeta 2^(1-zeta) exp(-50 eta) f_c(5)^2
    q = [[0, 0, 0], [5.0, 0, 0], [-5.0, 0, 0]]
    g4 = _G(_model("g4"), q, [1, 0, 0])
    m = _model()
    g5 = _G(m, q, [1, 0, 0])
    Fr = m.n_elements * m.n_rad
    assert np.all(g4[0, Fr:] == 0.0)
    for ie, eta in enumerate(m.ang_eta):
        for zeta in S.ZETAS:
            for lam in S.LAMBDAS:
                want = 2.0 ** (1 - zeta) * (1.0 - lam) ** zeta * math.exp(-50.0 * eta) * _fc(5.0) ** 2
                assert g5[0, _ang_index(m, 0, 0, ie, zeta, lam)] == pytest.approx(want, rel=1e-12, abs=1e-300)


def _addition_theorem_g5(m, d, species_nb):
    """G5 of one centre from its neighbour vectors d [K, 3] by the addition
    theorem: sum_{j in e1, k in e2} w_j w_k P_l(u_j . u_k)
    = 4 pi / (2l + 1) sum_m M_lm(e1) conj(M_lm(e2)), M_lm(e) = sum_{j in e} w_j Y_lm(u_j),
    with (1 + lambda c)^zeta expanded in Legendre polynomials."""
    r = np.linalg.norm(d, axis=1)
    polar = np.arccos(np.clip(d[:, 2] / r, -1.0, 1.0))
    azim = np.arctan2(d[:, 1], d[:, 0])
    fc = np.array([_fc(x) for x in r])
    Lmax = max(S.ZETAS)
    out = np.zeros(m.n_features)
    n_el = m.n_elements
    for ie, eta in enumerate(m.ang_eta):
        w = np.exp(-eta * r * r) * fc
        M = {}
        for e in range(n_el):
            sel = species_nb == e
            M[e] = [np.array([np.sum(w[sel] * special.sph_harm_y(l, mm, polar[sel], azim[sel]))
                              for mm in range(-l, l + 1)]) for l in range(Lmax + 1)]
        for e1 in range(n_el):
            for e2 in range(e1, n_el):
                Sl = np.array([4 * math.pi / (2 * l + 1) * np.real(np.sum(M[e1][l] * np.conj(M[e2][l])))
                               for l in range(Lmax + 1)])
                diag = np.sum(w[species_nb == e1] ** 2) if e1 == e2 else 0.0
                for zeta in S.ZETAS:
                    for lam in S.LAMBDAS:
                        poly = [math.comb(zeta, n) * lam ** n for n in range(zeta + 1)]
                        a = legendre.poly2leg(poly)
                        tot = float(np.dot(a, Sl[:len(a)]))
                        if e1 == e2:
                            tot = 0.5 * (tot - (1.0 + lam) ** zeta * diag)
                        out[_ang_index(m, e1, e2, ie, zeta, lam)] = 2.0 ** (1 - zeta) * tot
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_matches_spherical_harmonic_addition_theorem(seed):
    m = _model()
    rng = np.random.default_rng(seed)
    K = 24
    d = rng.uniform(-4.0, 4.0, size=(K, 3))
    d = d[np.linalg.norm(d, axis=1) > 0.8][:K]
    q = np.concatenate([[np.zeros(3)], d])
    species = np.concatenate([[1], rng.integers(0, 2, len(d))]).astype(np.int32)
    G = _G(m, q, species)
    want = _addition_theorem_g5(m, d, species[1:])
    Fr = m.n_elements * m.n_rad
    assert np.allclose(G[0, Fr:], want[Fr:], rtol=1e-10, atol=1e-12 * np.abs(want).max())


def test_equals_g4_when_the_r_jk_factors_are_one():
    # eta = 0 and a cutoff far beyond the cluster: exp(-eta r_jk^2) = 1 and
    # f_c(r_jk) = 1 - (pi r_jk / R_c)^2 / 4 + ..., so G4 and G5 agree to ~1e-11
    rc = 1.0e7
    base = S.make_model(["H", "O"], 4, 8, [16], 3)
    base = dataclasses.replace(base, cutoff=rc, ang_eta=np.array([0.0]))
    rng = np.random.default_rng(4)
    q = rng.uniform(-3.0, 3.0, size=(9, 3))
    species = rng.integers(0, 2, 9).astype(np.int32)
    start, idx = neighbors.brute_force_fp32(q.astype(np.float32), np.zeros(3), rc)
    centres = np.arange(9, dtype=np.int32)
    g4 = bpnn.descriptors(base, q, species, np.zeros(3), centres, start, idx)
    g5 = bpnn.descriptors(dataclasses.replace(base, angular="g5"), q, species, np.zeros(3), centres, start, idx)
    Fr = base.n_elements * base.n_rad
    assert np.abs(g5[:, Fr:]).max() > 1.0
    assert np.allclose(g5, g4, rtol=1e-10, atol=0.0)


def _energy(model, q, species, box, start, idx):
    G = bpnn.descriptors(model, q, species, box, np.arange(len(q)), start, idx)
    Ei, _ = bpnn.mlp_energy_grad(model, species, bpnn.normalise(model, G, species))
    return Ei.sum()


@pytest.mark.parametrize("kind", ["water8", "fad"])
def test_forces_central_fd(kind):
    wl = S.with_g5(S.small_workload(kind))
    s = wl.systems[0]
    q32 = S.perturbed_beads(wl, 0.05, seed=1)[: s.n_atoms]
    q = q32.astype(np.float64)
    E, F, W = bpnn.bead_energy_forces(wl.model, q32, s.species, s.box)
    start, idx = neighbors.brute_force_fp32(q32, s.box, RC)
    rng = np.random.default_rng(2)
    h = 1e-4
    worst = 0.0
    scale = np.sqrt(np.mean(F ** 2))
    for a in rng.choice(s.n_atoms, min(10, s.n_atoms), replace=False):
        for c in range(3):
            qp, qm = q.copy(), q.copy()
            qp[a, c] += h
            qm[a, c] -= h
            fd = -(_energy(wl.model, qp, s.species, s.box, start, idx)
                   - _energy(wl.model, qm, s.species, s.box, start, idx)) / (2 * h)
            worst = max(worst, abs(fd - F[a, c]) / scale)
    assert worst < 1e-6


def test_forces_sum_to_zero_and_torque_free():
    wl = S.with_g5(S.workload(1))
    s = wl.systems[0]
    q32 = S.perturbed_beads(wl, 0.05, seed=3)[: s.n_atoms]
    E, F, W = bpnn.bead_energy_forces(wl.model, q32, s.species, s.box)
    assert np.abs(F.sum(axis=0)).max() < 1e-12
    assert np.abs(np.cross(q32.astype(np.float64), F).sum(axis=0)).max() < 1e-12


def test_unknown_angular_form_is_rejected():
    m = _model("g6")
    with pytest.raises(ValueError):
        _G(m, [[0, 0, 0], [1.0, 0, 0]], [0, 0])
