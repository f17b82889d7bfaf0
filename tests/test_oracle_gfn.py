"""Pins of the direct-force head oracle (graph field network form, Sec. 2.2)
against properties the definition fixes: Newton's third law, rotation,
translation and permutation equivariance, edge symmetry, the pair-force
closed form of a constant readout, and a loop-by-loop evaluation on a tiny
system."""
import copy
import math

import numpy as np

from paper_2503_23728_amd import synthetic as S
from oracle import gfn


def _fad():
    wl = S.gfn_workload(1)
    s = wl.systems[0]
    return wl.model, s.q0.astype(np.float32), s.species, s.box


def _water():
    wl = S.gfn_workload(2)
    s = wl.systems[0]
    return wl.model, s.q0.astype(np.float32), s.species, s.box


def test_newton_third_law():
    for model, q, sp, box in (_fad(), _water()):
        F = gfn.bead_forces(model, q, sp, box)
        assert np.abs(F.sum(axis=0)).max() < 1e-12 * np.abs(F).sum()


def test_forces_are_central_sums_torque_free_for_a_molecule():
    model, q, sp, box = _fad()
    F = gfn.bead_forces(model, q, sp, box)
    torque = np.cross(q.astype(np.float64), F).sum(axis=0)
    assert np.abs(torque).max() < 1e-10 * np.abs(F).sum()


def test_edge_representations_are_symmetric():
    model, q, sp, box = _water()
    _, parts = gfn.bead_forces(model, q, sp, box, return_parts=True)
    key = {(int(i), int(j)): k for k, (i, j) in enumerate(zip(parts["owner"], parts["nbr"]))}
    for (i, j), k in list(key.items())[:500]:
        assert np.allclose(parts["e"][k], parts["e"][key[j, i]], rtol=0, atol=1e-12)


def test_rotation_equivariance():
    model, q, sp, box = _fad()
    rng = np.random.default_rng(4)
    A = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    F = gfn.bead_forces(model, q, sp, box)
    # rotate in FP64, then hand the rotated float32 positions to the head
    qr = (q.astype(np.float64) @ A.T).astype(np.float32)
    Fr = gfn.bead_forces(model, qr, sp, box)
    # the float32 rounding of the rotated positions (~1e-7 A) is the only difference
    assert np.abs(Fr - F @ A.T).max() < 1e-5 * np.abs(F).max()


def test_translation_invariance_periodic():
    model, q, sp, box = _water()
    F = gfn.bead_forces(model, q, sp, box)
    shift = np.array([0.37, -1.25, 2.5], dtype=np.float32)    # exact in float32 at these magnitudes
    F2 = gfn.bead_forces(model, q + shift, sp, box)
    assert np.abs(F2 - F).max() < 1e-5 * np.abs(F).max()


def test_permutation_equivariance():
    model, q, sp, box = _water()
    F = gfn.bead_forces(model, q, sp, box)
    rng = np.random.default_rng(5)
    perm = np.arange(len(sp))
    for e in np.unique(sp):
        idx = np.where(sp == e)[0]
        perm[idx] = rng.permutation(idx)
    Fp = gfn.bead_forces(model, q[perm], sp[perm], box)
    assert np.allclose(Fp, F[perm], rtol=0, atol=1e-10)


def test_constant_readout_is_a_cutoff_weighted_sum_of_unit_vectors():
    # phi_f = c everywhere (W1 = 0, b1 = 0, b2 = c): F_i = c sum_j f_c(r_ij) u_ij,
    # evaluated here straight from the geometry over all pairs
    model, q, sp, box = _water()
    m = copy.deepcopy(model)
    W1, b1, w2, _ = m.force
    c = 0.75     # exact in float32
    m.force = (np.zeros_like(W1), np.zeros_like(b1), w2, np.float32(c))
    F = gfn.bead_forces(m, q, sp, box)
    q64 = q.astype(np.float64)
    ref = np.zeros_like(F)
    for i in range(len(q)):
        d = q64 - q64[i]
        d -= box * np.round(d / box)
        r = np.sqrt((d * d).sum(axis=1))
        inside = (r > 0) & (r < m.cutoff)
        fc = 0.5 * (np.cos(np.pi * r[inside] / m.cutoff) + 1.0)
        ref[i] = c * ((fc / r[inside])[:, None] * d[inside]).sum(axis=0)
    assert np.abs(F - ref).max() < 1e-12 * np.abs(ref).max()


def _loop_forces(model, q, sp, box):
    """The same definitions evaluated edge by edge with Python loops."""
    n = len(q)
    q64 = np.asarray(q, dtype=np.float64)
    nb = {i: [] for i in range(n)}
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d = q64[j] - q64[i]
            if np.any(box > 0):
                d = d - box * np.round(d / box)
            r = math.sqrt(float(d @ d))
            if r < model.cutoff:
                nb[i].append((j, d, r))

    def phi(p, x):
        W1, b1, W2, b2 = (np.asarray(a, dtype=np.float64) for a in p)
        return W2 @ np.tanh(W1 @ x + b1) + b2

    e = {}
    for i in range(n):
        for j, d, r in nb[i]:
            fc = 0.5 * (math.cos(math.pi * r / model.cutoff) + 1.0)
            rho = np.array([math.exp(-eta * (r - Rs) ** 2) * fc for Rs, eta in zip(model.rad_center, model.rad_eta)])
            e[i, j] = np.asarray(model.edge_in, dtype=np.float64) @ rho + model.pair_embed[sp[i], sp[j]]
    node = [np.asarray(model.node_embed[sp[i]], dtype=np.float64) for i in range(n)]
    for msg, upd, edg in model.layers:
        new_node = []
        for i in range(n):
            m = sum((phi(msg, e[i, j]) for j, _, _ in nb[i]), np.zeros(model.width))
            new_node.append(node[i] + phi(upd, np.concatenate([node[i], m])))
        e = {(i, j): v + phi(edg, node[i] + node[j]) for (i, j), v in e.items()}
        node = new_node
    W1, b1, w2, b2 = (np.asarray(a, dtype=np.float64) for a in model.force)
    F = np.zeros((n, 3))
    for i in range(n):
        for j, d, r in nb[i]:
            fc = 0.5 * (math.cos(math.pi * r / model.cutoff) + 1.0)
            F[i] += fc * (w2 @ np.tanh(W1 @ e[i, j] + b1) + b2) * d / r
    return F


def test_matches_edge_by_edge_loops_on_a_small_system():
    model, q, sp, box = _fad()
    assert np.allclose(gfn.bead_forces(model, q, sp, box), _loop_forces(model, q, sp, box), rtol=1e-12, atol=1e-12)
    wl = S.small_workload("water8", n_beads=1)
    head = S.make_gfn_model(wl.model.elements, wl.model.n_rad, 16, 2, 77)
    s = wl.systems[0]
    q8 = s.q0.astype(np.float32)
    assert np.allclose(gfn.bead_forces(head, q8, s.species, s.box), _loop_forces(head, q8, s.species, s.box),
                       rtol=1e-12, atol=1e-12)
