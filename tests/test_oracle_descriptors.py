"""Pins of the oracle's neighbour sets, symmetry functions, network and forces.

Every expectation here comes from something other than the oracle itself:
closed forms for 2- and 3-atom geometries, a brute-force vs cell-list cross
check, central finite differences of the FP64 energy, symmetry invariances,
and a library (torch CPU autograd) evaluation of the per-element network.
"""
import math

import numpy as np
import pytest

from oracle import bpnn, neighbors
from paper_2503_23728_amd import synthetic as S

RC = 6.0


def _model(elements=("H", "O"), n_rad=16, n_ang=16, hidden=(32, 16), seed=5):
    return S.make_model(list(elements), n_rad, n_ang, list(hidden), seed)


def _fc(r):
    return 0.5 * (math.cos(math.pi * r / RC) + 1.0) if r < RC else 0.0


def _G(model, q, species, box=np.zeros(3)):
    q = np.asarray(q, dtype=np.float64)
    start, idx = neighbors.brute_force_fp32(q.astype(np.float32), box, model.cutoff)
    return bpnn.descriptors(model, q, np.asarray(species, np.int32), box, np.arange(len(q)), start, idx)


def _ang_index(model, e1, e2, ieta, zeta, lam):
    n_el = model.n_elements
    a, b = min(e1, e2), max(e1, e2)
    pair = a * n_el - a * (a - 1) // 2 + (b - a)
    iz = S.ZETAS.index(zeta)
    il = 0 if lam > 0 else 1
    return n_el * model.n_rad + pair * model.n_ang + (ieta * 4 + iz) * 2 + il


# ---------------------------------------------------------------- neighbours

def test_neighbors_cell_list_equals_brute_force_small_box():
    # 8 waters in a 12.5 A box: 2 cells per axis, the stencil wraps onto itself
    wl = S.small_workload("water8")
    s = wl.systems[0]
    rng = np.random.default_rng(3)
    q = (s.q0 + rng.normal(0, 0.3, s.q0.shape) + 40.0).astype(np.float32)   # far outside the box
    a = neighbors.brute_force_fp32(q, s.box, RC)
    b = neighbors.cell_list_fp32(q, s.box, RC)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_neighbors_cell_list_equals_brute_force_many_cells():
    rng = np.random.default_rng(4)
    box = np.array([19.5, 25.0, 31.0])          # 3, 4 and 5 cells per axis
    q = (rng.uniform(-1, 2, (700, 3)) * box).astype(np.float32)
    a = neighbors.brute_force_fp32(q, box, RC)
    b = neighbors.cell_list_fp32(q, box, RC)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_neighbors_match_fp64_set_and_are_symmetric():
    rng = np.random.default_rng(5)
    box = np.array([14.0, 14.0, 14.0])
    q = (rng.uniform(0, 1, (300, 3)) * box).astype(np.float32)
    start, idx = neighbors.brute_force_fp32(q, box, RC)
    dense = neighbors.csr_to_dense(start, idx, len(q))
    assert np.array_equal(dense, dense.T)
    m64, r2 = neighbors.fp64_pairs(q.astype(np.float64), box, RC)
    diff = dense != m64
    assert np.all(np.abs(r2[diff] - RC * RC) < 1e-4)
    # lists are sorted by (i, j)
    for i in range(len(q)):
        row = idx[start[i]:start[i + 1]]
        assert np.all(np.diff(row) > 0)


def test_neighbors_non_periodic_and_rejects_large_cutoff():
    q = np.array([[0, 0, 0], [5.9, 0, 0], [6.1, 0, 0], [0, 3, 4]], dtype=np.float32)
    start, idx = neighbors.brute_force_fp32(q, np.zeros(3), RC)
    assert list(idx[start[0]:start[1]]) == [1, 3]
    assert list(idx[start[2]:start[3]]) == [1]
    with pytest.raises(ValueError):
        neighbors.brute_force_fp32(q, np.array([11.0, 20.0, 20.0]), RC)


# ---------------------------------------------------------------- descriptors

def test_two_atom_radial_closed_form():
    m = _model()
    r = 2.3
    G = _G(m, [[0, 0, 0], [r, 0, 0]], [1, 0])          # O centre, H neighbour
    for s in range(m.n_rad):
        want = math.exp(-m.rad_eta[s] * (r - m.rad_center[s]) ** 2) * _fc(r)
        assert G[0, 0 * m.n_rad + s] == pytest.approx(want, rel=1e-12, abs=1e-300)
        assert G[0, 1 * m.n_rad + s] == 0.0             # no O neighbour
    assert np.all(G[:, m.n_elements * m.n_rad:] == 0.0)  # no triplet with two atoms


def test_two_atom_across_periodic_boundary():
    m = _model()
    box = np.array([13.0, 13.0, 13.0])
    G = _G(m, [[0.2, 6.0, 6.0], [12.5, 6.0, 6.0]], [1, 1], box)    # minimum image 0.7 A
    r = 0.7
    for s in range(m.n_rad):
        want = math.exp(-m.rad_eta[s] * (r - m.rad_center[s]) ** 2) * _fc(r)
        assert G[0, m.n_rad + s] == pytest.approx(want, rel=1e-9)


def test_three_atom_equilateral_angular_closed_form():
    # one triplet: cos theta = 1/2, all three distances a
    m = _model()
    a = 2.1
    q = [[0, 0, 0], [a, 0, 0], [a / 2, a * math.sqrt(3) / 2, 0]]
    G = _G(m, q, [1, 0, 0])       # O centre, two H neighbours -> block (H, H)
    for ie, eta in enumerate(m.ang_eta):
        for zeta in S.ZETAS:
            for lam in S.LAMBDAS:
                want = 2.0 ** (1 - zeta) * (1 + lam * 0.5) ** zeta * math.exp(-eta * 3 * a * a) * _fc(a) ** 3
                got = G[0, _ang_index(m, 0, 0, ie, zeta, lam)]
                assert got == pytest.approx(want, rel=1e-12)
    # the (H, O) and (O, O) blocks stay empty for the O centre
    assert G[0, _ang_index(m, 0, 1, 0, 1, 1.0)] == 0.0


def test_three_atom_right_angle_mixed_pair_block():
    # H centre at the corner of a right angle, O and H neighbours: cos = 0
    m = _model()
    b, c = 1.5, 2.5
    q = [[0, 0, 0], [b, 0, 0], [0, c, 0]]
    G = _G(m, q, [0, 1, 0])
    rjk = math.hypot(b, c)
    for ie, eta in enumerate(m.ang_eta):
        for zeta in S.ZETAS:
            for lam in S.LAMBDAS:
                want = 2.0 ** (1 - zeta) * math.exp(-eta * (b * b + c * c + rjk * rjk)) * _fc(b) * _fc(c) * _fc(rjk)
                assert G[0, _ang_index(m, 0, 1, ie, zeta, lam)] == pytest.approx(want, rel=1e-12)


def test_triplet_with_far_pair_contributes_nothing():
    # j and k both within R_c of i, but r_jk > R_c: f_c(r_jk) = 0
    m = _model()
    q = [[0, 0, 0], [5.0, 0, 0], [-5.0, 0, 0]]
    G = _G(m, q, [1, 0, 0])
    assert np.all(G[0, m.n_elements * m.n_rad:] == 0.0)
    assert np.any(G[0, :m.n_elements * m.n_rad] > 0)


# ---------------------------------------------------------------- network

def test_mlp_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    m = _model(hidden=(32, 24, 16))
    rng = np.random.default_rng(8)
    x = rng.normal(size=(40, m.n_features))
    sp = rng.integers(0, 2, 40).astype(np.int32)
    E, dx = bpnn.mlp_energy_grad(m, sp, x)
    for e in range(2):
        sel = sp == e
        xt = torch.tensor(x[sel], dtype=torch.float64, requires_grad=True)
        h = xt
        layers = m.weights[e]
        for W, b in layers[:-1]:
            h = torch.tanh(torch.nn.functional.linear(h, torch.tensor(W, dtype=torch.float64),
                                                      torch.tensor(b, dtype=torch.float64)))
        out = torch.nn.functional.linear(h, torch.tensor(layers[-1][0], dtype=torch.float64),
                                         torch.tensor(layers[-1][1], dtype=torch.float64))[:, 0]
        out.sum().backward()
        assert np.allclose(out.detach().numpy(), E[sel], rtol=1e-13, atol=1e-13)
        assert np.allclose(xt.grad.numpy(), dx[sel], rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- forces

def _energy(model, q, species, box, start, idx):
    G = bpnn.descriptors(model, q, species, box, np.arange(len(q)), start, idx)
    Ei, _ = bpnn.mlp_energy_grad(model, species, bpnn.normalise(model, G, species))
    return Ei.sum()


def test_forces_central_fd_water64():
    # 64 H2O (12.42 A box): central FD, h = 1e-4 A, 20 random atoms
    wl = S.workload(2)
    s = wl.systems[0]
    q32 = S.perturbed_beads(wl, 0.05, seed=1)[: s.n_atoms]
    q = q32.astype(np.float64)
    E, F, W = bpnn.bead_energy_forces(wl.model, q32, s.species, s.box)
    start, idx = neighbors.brute_force_fp32(q32, s.box, RC)
    rng = np.random.default_rng(2)
    h = 1e-4
    worst = 0.0
    scale = np.sqrt(np.mean(F ** 2))
    for a in rng.choice(s.n_atoms, 20, replace=False):
        for c in range(3):
            qp, qm = q.copy(), q.copy()
            qp[a, c] += h
            qm[a, c] -= h
            fd = -(_energy(wl.model, qp, s.species, s.box, start, idx)
                   - _energy(wl.model, qm, s.species, s.box, start, idx)) / (2 * h)
            worst = max(worst, abs(fd - F[a, c]) / scale)
    assert worst < 1e-6


def test_virial_matches_strain_fd():
    wl = S.small_workload("water8")
    s = wl.systems[0]
    q32 = S.perturbed_beads(wl, 0.05, seed=2)[: s.n_atoms]
    q = q32.astype(np.float64)
    E, F, W = bpnn.bead_energy_forces(wl.model, q32, s.species, s.box)
    start, idx = neighbors.brute_force_fp32(q32, s.box, RC)
    # energy under the affine strain d_ij -> (1 + eps) d_ij of every neighbour vector
    h = 1e-6
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3))
            eps[a, b] = h
            dE = (_sheared_energy(wl.model, q, s.species, s.box, start, idx, eps)
                  - _sheared_energy(wl.model, q, s.species, s.box, start, idx, -eps)) / (2 * h)
            # W_ab = -sum d_a dE/dd_b = -dE/deps_ba; the virial is symmetric
            assert -dE == pytest.approx(W[b, a], rel=1e-6, abs=1e-8 * np.abs(W).max())
    assert np.allclose(W, W.T, rtol=1e-9, atol=1e-12 * np.abs(W).max())


def _sheared_energy(model, q, species, box, start, idx, eps):
    """Energy with every neighbour vector d_ij replaced by (1+eps) d_ij (the
    reference minimum image kept), built as a non-periodic cluster per centre."""
    n = len(q)
    E = 0.0
    for i in range(n):
        nb = idx[start[i]:start[i + 1]]
        d = q[nb] - q[i]
        d = d - box * np.round(d / box)
        d = d @ (np.eye(3) + eps).T
        local = np.concatenate([[np.zeros(3)], d])
        sp = np.concatenate([[species[i]], species[nb]]).astype(np.int32)
        cs = np.array([0, len(nb)], dtype=np.int64)
        G = bpnn.descriptors(model, local, sp, np.zeros(3), np.array([0]), cs, np.arange(1, len(nb) + 1))
        Ei, _ = bpnn.mlp_energy_grad(model, sp[:1], bpnn.normalise(model, G, sp[:1]))
        E += Ei[0]
    return E


def test_forces_sum_to_zero_and_torque_free():
    wl = S.workload(1)
    s = wl.systems[0]
    q32 = S.perturbed_beads(wl, 0.05, seed=3)[: s.n_atoms]
    E, F, W = bpnn.bead_energy_forces(wl.model, q32, s.species, s.box)
    assert np.abs(F.sum(axis=0)).max() < 1e-12
    torque = np.cross(q32.astype(np.float64), F).sum(axis=0)
    assert np.abs(torque).max() < 1e-12


def test_energy_invariances():
    wl = S.workload(1)
    s = wl.systems[0]
    q = S.perturbed_beads(wl, 0.05, seed=4)[: s.n_atoms].astype(np.float64)
    E0, _, _ = bpnn.bead_energy_forces(wl.model, q.astype(np.float32), s.species, s.box)
    # rotation + translation (float32 inputs: compare at float32 input precision)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    R = R @ np.array([[1, 0, 0], [0, math.cos(1.1), -math.sin(1.1)], [0, math.sin(1.1), math.cos(1.1)]])
    q2 = q @ R.T + np.array([1.5, -2.0, 0.25])
    E1, _, _ = bpnn.bead_energy_forces(wl.model, q2.astype(np.float32), s.species, s.box)
    assert E1 == pytest.approx(E0, rel=1e-5)
    # permutation of same-element atoms is exact
    perm = np.arange(s.n_atoms)
    h = np.nonzero(s.species == 0)[0]
    perm[h] = h[::-1]
    E2, _, _ = bpnn.bead_energy_forces(wl.model, q[perm].astype(np.float32), s.species[perm], s.box)
    assert E2 == pytest.approx(E0, rel=1e-12)


def test_periodic_translation_invariance():
    wl = S.small_workload("water8")
    s = wl.systems[0]
    q32 = S.perturbed_beads(wl, 0.05, seed=5)[: s.n_atoms]
    q = q32.astype(np.float64)
    start, idx = neighbors.brute_force_fp32(q32, s.box, RC)
    E0 = _energy(wl.model, q, s.species, s.box, start, idx)
    # whole box lengths per atom (different per atom) leave every minimum image unchanged
    rng = np.random.default_rng(6)
    shift = rng.integers(-3, 4, size=q.shape) * s.box
    E1 = _energy(wl.model, q + shift, s.species, s.box, start, idx)
    assert E1 == pytest.approx(E0, rel=1e-12)
