"""Pins of the well-tempered metadynamics oracle (Sec. 2.5; CVs of Sec. 3.1,
Sec. 3.2) against what geometry and mathematics fix, independently of the
oracle's own formulas:

* s_dimer of the constructed dimer is -1.48 A (O...O 2.70 A, O-H 0.98 A on
  the O...O line) and +1.48 A with both protons moved across.
* The XRD CV equals the orientational average of the scattered intensity
  |sum_j f_j exp(i q . r_j)|^2 / N over directions of q at |q| = Q (Debye's
  derivation of the sinc sum), computed by quadrature on the sphere; and it
  reduces to closed forms for one atom, two atoms and Q -> 0.
* Gradients of both CVs and of the bias agree with central differences;
  the CVs are invariant under translation, rotation and permutation, and the
  periodic XRD sum is invariant under moving an atom by a box vector.
* Well-tempered deposition on a 1-D double well converges to
  V(s) = -(1 - 1/gamma) F(s) + const (the convergence statement of
  Sec. 2.5), and with gamma -> infinity every hill has the initial height.
* The path-integral reweighting reduces to the bead free energy when all
  beads share one bias, and to the two-term closed form for P = 2.
"""
import math

import numpy as np
import pytest

from oracle import metad
from oracle.constants import KB
from paper_2503_23728_amd import synthetic as S


def _rot(rng):
    A = rng.normal(size=(3, 3))
    Q, R = np.linalg.qr(A)
    return Q * np.sign(np.diag(R))[None, :]


def test_s_dimer_of_the_constructed_dimer():
    _, _, pos = S.formic_acid_dimer()
    s, _ = metad.cv_distances(pos, np.zeros(3), S.FAD_DPT_ATOMS, S.FAD_DPT_COEF)
    assert s == pytest.approx(-1.48, abs=1e-12)
    # move each hydroxyl proton to 0.98 A from the acceptor oxygen on the same line
    moved = pos.copy()
    for h, donor, acc in ((4, 2, 6), (9, 7, 1)):
        u = (pos[acc] - pos[donor]) / np.linalg.norm(pos[acc] - pos[donor])
        moved[h] = pos[acc] - 0.98 * u
    s2, _ = metad.cv_distances(moved, np.zeros(3), S.FAD_DPT_ATOMS, S.FAD_DPT_COEF)
    assert s2 == pytest.approx(1.48, abs=1e-12)


def _fd_grad(fn, q, h=1e-5):
    g = np.zeros_like(q)
    for i in range(len(q)):
        for c in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, c] += h
            qm[i, c] -= h
            g[i, c] = (fn(qp) - fn(qm)) / (2 * h)
    return g


@pytest.mark.parametrize("periodic", [False, True])
def test_distance_cv_gradient_matches_central_differences(periodic):
    rng = np.random.default_rng(1)
    box = np.array([5.0, 6.0, 7.0]) if periodic else np.zeros(3)
    q = rng.uniform(0, 5, size=(8, 3))
    atoms = np.array([[0, 1], [2, 1], [3, 7], [5, 6], [0, 7]])
    coef = np.array([1.0, -1.0, 0.5, 2.0, -0.7])
    _, g = metad.cv_distances(q, box, atoms, coef)
    g_fd = _fd_grad(lambda x: metad.cv_distances(x, box, atoms, coef)[0], q)
    assert np.max(np.abs(g - g_fd)) < 1e-8


def _sphere_average(fn, n_theta=64, n_phi=128):
    """Average of fn(unit vectors [M, 3]) over the sphere: Gauss-Legendre in
    cos(theta) times the trapezoid rule in phi (exact for spherical
    harmonics up to degree 2 n_theta - 1 in theta and n_phi - 1 in phi)."""
    x, w = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1 - x * x)
    u = np.stack([st[:, None] * np.cos(phi)[None, :], st[:, None] * np.sin(phi)[None, :],
                  np.broadcast_to(x[:, None], (n_theta, n_phi))], axis=-1).reshape(-1, 3)
    vals = fn(u).reshape(n_theta, n_phi)
    return float(np.sum(w[:, None] * vals) / (2 * n_phi))


def test_xrd_cv_is_the_orientational_average_of_the_intensity():
    rng = np.random.default_rng(2)
    n = 9
    q = rng.uniform(-1.5, 1.5, size=(n, 3))
    species = rng.integers(0, 2, size=n)
    f = np.array([0.69, 6.7])
    Q = 1.69
    S_cv, _ = metad.cv_xrd(q, species, np.zeros(3), Q, f)
    fa = f[species]

    def intensity(u):
        phase = Q * (u @ q.T)                       # [M, n]
        amp = (fa[None, :] * np.exp(1j * phase)).sum(axis=1)
        return np.abs(amp) ** 2 / n
    assert S_cv == pytest.approx(_sphere_average(intensity), rel=1e-10)


def test_xrd_cv_closed_forms():
    f = np.array([0.7, 6.7])
    Q = 1.69
    one, _ = metad.cv_xrd(np.zeros((1, 3)), [1], np.zeros(3), Q, f)
    assert one == pytest.approx(6.7 ** 2, rel=1e-14)
    R = 1.3
    two, g = metad.cv_xrd(np.array([[0.0, 0, 0], [R, 0, 0]]), [0, 1], np.zeros(3), Q, f)
    x = Q * R
    assert two == pytest.approx(0.5 * (0.7 ** 2 + 6.7 ** 2 + 2 * 0.7 * 6.7 * math.sin(x) / x), rel=1e-14)
    # dS/dx_2 = (1/2) 2 f1 f2 Q d/dx sinc(x) for the pair along x
    assert g[1, 0] == pytest.approx(0.7 * 6.7 * Q * (x * math.cos(x) - math.sin(x)) / (x * x), rel=1e-12)
    assert g[0, 0] == pytest.approx(-g[1, 0], rel=1e-14)
    rng = np.random.default_rng(3)
    q = rng.uniform(0, 3, size=(6, 3))
    sp = rng.integers(0, 2, size=6)
    small, _ = metad.cv_xrd(q, sp, np.zeros(3), 1e-7, f)
    assert small == pytest.approx(np.sum(f[sp]) ** 2 / 6, rel=1e-12)


@pytest.mark.parametrize("periodic", [False, True])
def test_xrd_gradient_and_invariances(periodic):
    rng = np.random.default_rng(4)
    n = 10
    box = np.array([6.0, 7.0, 8.0]) if periodic else np.zeros(3)
    q = rng.uniform(0, 6, size=(n, 3))
    sp = rng.integers(0, 2, size=n)
    f = np.array([0.69, 6.73])
    Q = 1.69
    S0, g = metad.cv_xrd(q, sp, box, Q, f)
    g_fd = _fd_grad(lambda x: metad.cv_xrd(x, sp, box, Q, f)[0], q)
    assert np.max(np.abs(g - g_fd)) < 1e-7
    assert np.max(np.abs(g.sum(axis=0))) < 1e-12          # translation invariance
    perm = rng.permutation(n)
    assert metad.cv_xrd(q[perm], sp[perm], box, Q, f)[0] == pytest.approx(S0, rel=1e-13)
    assert metad.cv_xrd(q + np.array([0.3, -1.1, 2.2]), sp, box, Q, f)[0] == pytest.approx(S0, rel=1e-13)
    if periodic:
        moved = q.copy()
        moved[3] += box * np.array([1, -2, 1])
        assert metad.cv_xrd(moved, sp, box, Q, f)[0] == pytest.approx(S0, rel=1e-13)
    else:
        R = _rot(rng)
        assert metad.cv_xrd(q @ R.T, sp, box, Q, f)[0] == pytest.approx(S0, rel=1e-13)
        s_d, _ = metad.cv_distances(q, box, [[0, 1], [2, 5]], [1.0, -1.0])
        assert metad.cv_distances(q @ R.T, box, [[0, 1], [2, 5]], [1.0, -1.0])[0] == pytest.approx(s_d, rel=1e-13)


def test_bias_shape_and_derivative():
    c = np.array([0.1, 0.5, -0.3])
    h = np.array([0.01, 0.02, 0.005])
    sig = 0.2
    v, _ = metad.bias(0.5, [0.5], [0.02], sig)
    assert v == pytest.approx(0.02, rel=1e-15)
    v, _ = metad.bias(0.5 + sig, [0.5], [0.02], sig)
    assert v == pytest.approx(0.02 * math.exp(-0.5), rel=1e-14)
    for s in (-0.7, 0.0, 0.33, 1.2):
        dfd = (metad.bias(s + 1e-6, c, h, sig)[0] - metad.bias(s - 1e-6, c, h, sig)[0]) / 2e-6
        assert metad.bias(s, c, h, sig)[1] == pytest.approx(dfd, rel=1e-7, abs=1e-12)
    assert metad.bias(0.3, [], [], sig) == (0.0, 0.0)


def test_infinite_bias_factor_gives_plain_metadynamics():
    assert metad.well_tempered_height(5.0, 300.0, 0.0104, math.inf) == 0.0104
    assert metad.well_tempered_height(0.0, 300.0, 0.0104, 10.0) == 0.0104


def test_well_tempered_bias_converges_to_scaled_free_energy():
    # overdamped Langevin in U(s) = a (s^2 - 1)^2 (barrier 4 kT) with the CV
    # s itself.  The converged bias is V = -(1 - 1/gamma) U + const; with
    # gamma = 2 the fitted slope is 1/2, where a height rule with gamma in
    # place of gamma - 1 would give 2/3 and plain metadynamics 1.
    rng = np.random.default_rng(5)
    T = 300.0
    kT = KB * T
    a, gamma, w0, sig = 4 * kT, 2.0, 0.2 * kT, 0.1
    D, dt, stride, n_steps = 1.0, 2e-3, 25, 100000
    centers, heights = [], []
    s = -1.0
    noise = rng.normal(size=n_steps)
    for step in range(1, n_steps + 1):
        _, dv = metad.bias(s, centers, heights, sig)
        s += D * (-4 * a * s * (s * s - 1) - dv) / kT * dt + math.sqrt(2 * D * dt) * noise[step - 1]
        if step % stride == 0:
            v_here, _ = metad.bias(s, centers, heights, sig)
            centers.append(s)
            heights.append(metad.well_tempered_height(v_here, T, w0, gamma))
    grid = np.linspace(-1.2, 1.2, 25)
    V = np.array([metad.bias(x, centers, heights, sig)[0] for x in grid])
    U = a * (grid ** 2 - 1) ** 2
    lam = np.linalg.lstsq(np.stack([-U, np.ones_like(U)], 1), V, rcond=None)[0][0]
    assert abs(lam - (1 - 1 / gamma)) < 0.05, lam
    # the heights decay as the bias fills the wells
    assert heights[-1] < 0.1 * w0


def test_quantum_reweighting_special_cases():
    rng = np.random.default_rng(6)
    grid = np.linspace(-1, 1, 11)
    c = list(rng.normal(0, 0.5, 20))
    h = list(rng.uniform(0.001, 0.01, 20))
    sig, gamma, T = 0.2, 10.0, 300.0
    same = metad.fes_quantum(grid, [c] * 4, [h] * 4, sig, gamma, T)
    one = np.array([-(gamma / (gamma - 1)) * metad.bias(x, c, h, sig)[0] for x in grid])
    np.testing.assert_allclose(same, one, rtol=1e-12, atol=1e-15)
    c2 = list(rng.normal(0, 0.5, 20))
    two = metad.fes_quantum(grid, [c, c2], [h, h], sig, gamma, T)
    F1 = one
    F2 = np.array([-(gamma / (gamma - 1)) * metad.bias(x, c2, h, sig)[0] for x in grid])
    beta = 1 / (KB * T)
    np.testing.assert_allclose(two, -np.log(0.5 * (np.exp(-beta * F1) + np.exp(-beta * F2))) / beta,
                               rtol=1e-12, atol=1e-15)


def test_deposition_uses_the_bias_before_the_hill_and_per_bead_histories():
    # two beads of one system; each bead's hills follow its own CV
    sys_ = [(2, 2, 300.0, np.array([0, 0]), np.zeros(3))]
    m = metad.Metad(sys_, ("distances", [[0, 1]], [1.0]), 0.01, 0.1, 5.0, 1)
    q = np.array([[0, 0, 0], [1.0, 0, 0], [0, 0, 0], [1.5, 0, 0]])
    fn = m.force_fn(lambda x: (np.zeros(2), np.zeros_like(x)))
    fn(q)
    m.deposit()
    fn(q)
    m.deposit()
    kT = KB * 300.0
    assert m.centers[0] == [1.0, 1.0] and m.centers[1] == [1.5, 1.5]
    assert m.heights[0][0] == 0.01
    assert m.heights[0][1] == pytest.approx(0.01 * math.exp(-0.01 / (kT * 4)), rel=1e-14)
    # bias force on the pair pulls along the CV gradient: zero at the hill centre
    _, _, F = m.bias_forces(q)
    assert np.max(np.abs(F)) < 1e-15


def test_form_factors_at_zero_angle_count_electrons():
    for e, Z in (("H", 1), ("C", 6), ("O", 8)):
        assert S.scattering_factor(e, 0.0) == pytest.approx(Z, abs=2e-3)
    assert S.scattering_vector(11.95, 1.54) == pytest.approx(1.68959, abs=1e-5)
