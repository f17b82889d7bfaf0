"""Pins of the oracle's normal modes, PILE-L integrator, estimators, Philox
noise and quantum-harmonic-oscillator closed forms.

Expectations come from outside the oracle: orthonormality and the spring
identity of the normal-mode matrix, numpy's real FFT, exact energy
conservation of the free ring polymer, a textbook velocity-Verlet loop for
P = 1, the dt^2 scaling of the NVE error, the exact finite-P harmonic
averages (Sec. S1) sampled by the thermostat, and moments of the noise.
"""
import json
import os

import numpy as np
import pytest

from oracle import philox, qho, ring

import ring_linear
from oracle.constants import KB, HBAR, MVV2E

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- normal modes

@pytest.mark.parametrize("P", [1, 2, 4, 6, 8, 32, 64, 128])
def test_nm_matrix_orthonormal(P):
    C = ring.nm_matrix(P)
    assert np.allclose(C.T @ C, np.eye(P), atol=1e-13)


@pytest.mark.parametrize("P", [2, 4, 8, 10, 32])
def test_nm_matrix_is_the_real_fft(P):
    rng = np.random.default_rng(P)
    q = rng.normal(size=P)
    qt = ring.nm_matrix(P).T @ q
    X = np.fft.rfft(q)                       # X_m = sum_j q_j exp(-2 pi i j m / P)
    want = np.empty(P)
    want[0] = X[0].real / np.sqrt(P)
    for m in range(1, P // 2):
        want[m] = np.sqrt(2.0 / P) * X[m].real
        want[P - m] = np.sqrt(2.0 / P) * X[m].imag    # column P-m is -sin(2 pi j m/P), as is Im X_m
    want[P // 2] = X[P // 2].real / np.sqrt(P)
    assert np.allclose(qt, want, atol=1e-12)


@pytest.mark.parametrize("P", [2, 8, 32])
def test_spring_energy_is_diagonal_in_normal_modes(P):
    rng = np.random.default_rng(1)
    m, T = 1.008, 300.0
    q = rng.normal(size=(P, 3))
    wk, wP = ring.mode_frequencies(P, T)
    bead = 0.5 * m * wP ** 2 * np.sum((np.roll(q, -1, axis=0) - q) ** 2)
    qt = ring.nm_matrix(P).T @ q
    mode = 0.5 * m * np.sum(wk[:, None] ** 2 * qt ** 2)
    assert mode == pytest.approx(bead, rel=1e-12)


# ---------------------------------------------------------------- integrator

def _systems(n, P, T, mass=1.008):
    return [(n, P, T, np.full(n, mass))]


def _hamiltonian(rp, V):
    est = rp.estimators()[0]
    return est["K_beads"] + est["E_spring"] + V


def test_free_ring_polymer_conserves_energy():
    # V = 0, thermostat off: the A step is exact, so H_P is conserved to rounding
    systems = _systems(5, 16, 300.0)
    rp = ring.RingPolymers(systems, 0.5, 0.0, 1.0, 1, lambda q: (np.zeros(16), np.zeros_like(q)))
    rng = np.random.default_rng(2)
    rp.set_state(rng.normal(0, 0.1, (80, 3)), rng.normal(0, 1.0, (80, 3)))
    h0 = _hamiltonian(rp, 0.0)
    for _ in range(500):
        rp.step()
    assert _hamiltonian(rp, 0.0) == pytest.approx(h0, rel=1e-11)


def test_single_bead_nve_is_velocity_verlet():
    omega = 0.02
    systems = _systems(4, 1, 300.0, mass=15.999)
    fn = ring.harmonic_force_fn(systems, omega)
    rp = ring.RingPolymers(systems, 0.5, 0.0, 1.0, 1, fn)
    rng = np.random.default_rng(3)
    q0, p0 = rng.normal(0, 0.2, (4, 3)), rng.normal(0, 1.0, (4, 3))
    rp.set_state(q0, p0)
    for _ in range(200):
        rp.step()
    # textbook velocity Verlet: kick, drift, force, kick
    m, k = 15.999, 15.999 * omega ** 2 * MVV2E
    q, p = q0.copy(), p0.copy()
    f = -k * q
    for _ in range(200):
        p = p + 0.25 * f / MVV2E
        q = q + 0.5 * p / m
        f = -k * q
        p = p + 0.25 * f / MVV2E
    assert np.allclose(rp.q, q, rtol=1e-12, atol=1e-14)
    assert np.allclose(rp.p, p, rtol=1e-12, atol=1e-14)


def test_nve_energy_error_scales_as_dt_squared():
    omega = 0.05
    P = 8
    systems = _systems(3, P, 300.0)
    errs = []
    for dt in (0.5, 0.25):
        fn = ring.harmonic_force_fn(systems, omega)
        rp = ring.RingPolymers(systems, dt, 0.0, 1.0, 1, fn)
        rng = np.random.default_rng(4)
        rp.set_state(rng.normal(0, 0.1, (P * 3, 3)), rng.normal(0, 3.0, (P * 3, 3)))
        h0 = rp.estimators()[0]["H_conserved"]
        worst = 0.0
        for _ in range(int(100 / dt)):
            rp.step()
            worst = max(worst, abs(rp.estimators()[0]["H_conserved"] - h0))
        errs.append(worst)
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5


def test_thermostat_heat_balances_energy():
    # with the thermostat on, H_P + heat stays constant up to the integration error
    omega = 0.02
    systems = _systems(6, 8, 300.0)
    fn = ring.harmonic_force_fn(systems, omega)
    rp = ring.RingPolymers(systems, 0.25, 50.0, 1.0, 9, fn)
    rng = np.random.default_rng(5)
    rp.set_state(rng.normal(0, 0.1, (48, 3)), rng.normal(0, 1.0, (48, 3)))
    h0 = rp.estimators()[0]["H_conserved"]
    for _ in range(400):
        rp.step()
    est = rp.estimators()[0]
    assert abs(est["heat_bath"]) > 1e-3
    assert abs(est["H_conserved"] - h0) < 1e-3 * abs(est["heat_bath"])


def test_single_bead_estimators_are_classical():
    systems = _systems(4, 1, 250.0)
    fn = ring.harmonic_force_fn(systems, 0.03)
    rp = ring.RingPolymers(systems, 0.5, 100.0, 1.0, 3, fn)
    rng = np.random.default_rng(6)
    rp.set_state(rng.normal(0, 0.1, (4, 3)), rng.normal(0, 1.0, (4, 3)))
    rp.step()
    est = rp.estimators()[0]
    assert est["E_spring"] == 0.0
    assert est["K_prim"] == pytest.approx(1.5 * 4 * KB * 250.0, rel=1e-14)
    assert est["K_cv"] == pytest.approx(1.5 * 4 * KB * 250.0, rel=1e-14)


def _block_mean(x, nblocks=20):
    b = np.array_split(np.asarray(x), nblocks)
    means = np.array([v.mean() for v in b])
    return means.mean(), means.std(ddof=1) / np.sqrt(nblocks)


@pytest.mark.parametrize("P", [1, 4, 8])
def test_pile_l_samples_exact_finite_P_harmonic_average(P):
    # Sec. S1 oscillator: many independent atoms in one ring polymer system
    g = json.load(open(os.path.join(GOLDEN, "qho_s1.json")))
    m, w = g["mass_amu"], g["omega_per_fs"]
    T = 100.0                                   # beta hbar w = 0.95: P = 8 far from classical and quantum
    n = 600
    systems = _systems(n, P, T, mass=m)
    rp = ring.RingPolymers(systems, g["dt_fs"], 100.0, 1.0, 17, ring.harmonic_force_fn(systems, w))
    rng = np.random.default_rng(7)
    rp.set_state(rng.normal(0, 0.3, (n * P, 3)), rng.normal(0, 0.2, (n * P, 3)))
    for _ in range(1500):
        rp.step()
    x2, kcv, kprim = [], [], []
    for t in range(3000):
        rp.step()
        if t % 5 == 0:
            x2.append(np.mean(rp.q ** 2))
            est = rp.estimators()[0]
            kcv.append(est["K_cv"] / (3 * n))
            kprim.append(est["K_prim"] / (3 * n))
    mean, err = _block_mean(x2)
    want = qho.x2_beads_sum(m, w, T, P)
    assert abs(mean - want) < 3.5 * err + 2e-3 * want
    # virial (centroid) kinetic energy = half the harmonic energy per dimension
    kmean, kerr = _block_mean(kcv)
    assert abs(kmean - 0.5 * qho.energy_beads(m, w, T, P)) < 3.5 * kerr + 2e-3 * kmean
    # primitive estimator: the same mean, K_prim = 3nP/(2 beta) - E_spring/P
    pmean, perr = _block_mean(kprim)
    assert abs(pmean - 0.5 * qho.energy_beads(m, w, T, P)) < 3.5 * perr + 2e-3 * pmean


def test_bead_temperature_is_P_times_T():
    P, n, T = 8, 800, 200.0
    systems = _systems(n, P, T)
    rp = ring.RingPolymers(systems, 0.5, 20.0, 1.0, 23, ring.harmonic_force_fn(systems, 0.01))
    rp.set_state(np.zeros((n * P, 3)), np.zeros((n * P, 3)))
    temps = []
    for t in range(600):
        rp.step()
        if t > 200:
            temps.append(rp.estimators()[0]["T_beads"])
    mean, err = _block_mean(temps)
    assert abs(mean - P * T) < 3.5 * err + 5e-3 * P * T


# ---------------------------------------------------------------- PILE-G and the centroid-virial pressure

def test_pile_g_centroid_kinetic_energy_relaxes_at_the_half_step_rate():
    # Bussi, Donadio, Parrinello (2007): over a half step, E[K'] = c K + (1 - c) Kbar,
    # c = exp(-(dt/2)/tau0), Kbar = N_f k_B T P / 2 -- averaged over the noise
    n, P, T, dt, tau0 = 5, 4, 300.0, 0.5, 2.0
    m = np.linspace(1.0, 16.0, n)
    rp = ring.RingPolymers([(n, P, T, m)], dt, tau0, 1.0, 1, lambda q: (np.zeros(P), np.zeros_like(q)),
                           thermostat="pile-g")
    rng = np.random.default_rng(30)
    p0 = rng.normal(size=(n, 3)) * np.sqrt(m)[:, None]
    kbar = 0.5 * 3 * n * KB * T * P
    K = 0.5 * MVV2E * np.sum(p0 * p0 / m[:, None])
    p0 *= np.sqrt(3.0 * kbar / K)                       # K = 3 Kbar
    K = 3.0 * kbar
    a2 = np.array([rp._svr_factor(0, p0, rng.normal(size=(n, 3))) ** 2 for _ in range(40000)])
    c = np.exp(-0.5 * dt / tau0)
    want = c + (1.0 - c) * kbar / K
    assert abs(a2.mean() - want) < 4 * a2.std() / np.sqrt(len(a2))
    # a full-step rate exp(-dt/tau0) is ruled out
    c2 = np.exp(-dt / tau0)
    assert abs(a2.mean() - (c2 + (1.0 - c2) * kbar / K)) > 10 * a2.std() / np.sqrt(len(a2))


@pytest.mark.parametrize("P", [1, 4])
def test_pile_g_samples_the_canonical_centroid_kinetic_energy(P):
    # free ring polymers: the centroid kinetic energy is touched only by the
    # global thermostat, whose stationary law is Gamma(N_f / 2, k_B T P) at any dt
    n, T = 4, 200.0
    m = np.array([1.0, 2.0, 12.0, 16.0])
    rp = ring.RingPolymers([(n, P, T, m)], 0.5, 3.0, 1.0, 31 + P, lambda q: (np.zeros(P), np.zeros_like(q)),
                           thermostat="pile-g")
    rng = np.random.default_rng(32)
    rp.set_state(np.zeros((n * P, 3)), rng.normal(size=(n * P, 3)))
    C = ring.nm_matrix(P)
    ks = []
    for t in range(12000):
        rp.step()
        if t >= 200:
            pt0 = np.einsum("j,jnc->nc", C[:, 0], rp.p.reshape(P, n, 3))
            ks.append(0.5 * MVV2E * np.sum(pt0 * pt0 / m[:, None]))
    ks = np.array(ks) / (KB * T * P)                    # in units of k_B T P: Gamma(6, 1)
    nf = 3 * n
    mean, err = _block_mean(ks, 40)
    assert abs(mean - nf / 2) < 4 * err
    var, verr = _block_mean((ks - nf / 2) ** 2, 40)
    assert abs(var - nf / 2) < 4 * verr                 # Gamma(k, 1): variance k
    skew, serr = _block_mean((ks - nf / 2) ** 3, 40)
    assert abs(skew - 2 * nf / 2) < 4 * serr            # third central moment 2k


def test_pile_g_samples_exact_finite_P_harmonic_average():
    g = json.load(open(os.path.join(GOLDEN, "qho_s1.json")))
    m, w = g["mass_amu"], g["omega_per_fs"]
    T, P, n = 100.0, 8, 600
    systems = _systems(n, P, T, mass=m)
    rp = ring.RingPolymers(systems, g["dt_fs"], 100.0, 1.0, 33, ring.harmonic_force_fn(systems, w),
                           thermostat="pile-g")
    rng = np.random.default_rng(34)
    rp.set_state(rng.normal(0, 0.3, (n * P, 3)), rng.normal(0, 0.2, (n * P, 3)))
    for _ in range(1500):
        rp.step()
    x2, kcv = [], []
    for t in range(3000):
        rp.step()
        if t % 5 == 0:
            x2.append(np.mean(rp.q ** 2))
            kcv.append(rp.estimators()[0]["K_cv"] / (3 * n))
    mean, err = _block_mean(x2)
    want = qho.x2_beads_sum(m, w, T, P)
    assert abs(mean - want) < 3.5 * err + 2e-3 * want
    kmean, kerr = _block_mean(kcv)
    assert abs(kmean - 0.5 * qho.energy_beads(m, w, T, P)) < 3.5 * kerr + 2e-3 * kmean


def test_pile_g_heat_balances_energy():
    omega = 0.02
    systems = _systems(6, 8, 300.0)
    rp = ring.RingPolymers(systems, 0.25, 50.0, 1.0, 35, ring.harmonic_force_fn(systems, omega),
                           thermostat="pile-g")
    rng = np.random.default_rng(36)
    rp.set_state(rng.normal(0, 0.1, (48, 3)), rng.normal(0, 1.0, (48, 3)))
    h0 = rp.estimators()[0]["H_conserved"]
    for _ in range(400):
        rp.step()
    est = rp.estimators()[0]
    assert abs(est["heat_bath"]) > 1e-3
    assert abs(est["H_conserved"] - h0) < 1e-3 * abs(est["heat_bath"])


def test_pressure_of_free_ring_polymers_is_the_ideal_gas_law():
    n, P, T = 7, 8, 250.0
    box = np.array([10.0, 12.0, 9.0])
    rp = ring.RingPolymers([(n, P, T, np.full(n, 2.0))], 0.5, 100.0, 1.0, 3,
                           lambda q: (np.zeros(P), np.zeros_like(q), np.zeros((P, 3, 3))), boxes=[box])
    rng = np.random.default_rng(37)
    rp.set_state(rng.normal(0, 2.0, (n * P, 3)), rng.normal(size=(n * P, 3)))
    assert rp.estimators()[0]["P_cv"] == pytest.approx(n * KB * T / np.prod(box), rel=1e-13)


def test_centroid_virial_pressure_is_minus_the_free_energy_strain_derivative():
    # P_cv V - N k_B T = -(1/3) d/de (1/P) sum_k E(q^k(e)) at e = 0, where the
    # box and the centroids scale by (1 + e) and every bead keeps its offset
    # from its centroid; central differences of the FP64 oracle energy
    from paper_2503_23728_amd import synthetic as S
    from oracle import bpnn, neighbors
    wl = S.small_workload("water8", n_beads=4)
    s = wl.systems[0]
    P, n = s.n_beads, s.n_atoms
    q = S.perturbed_beads(wl, 0.08, seed=38).astype(np.float64)
    rp = ring.RingPolymers([(n, P, s.temperature, wl.model.masses[s.species])], wl.dt, wl.tau0, 1.0, 1,
                           lambda qq: bpnn.energy_forces(wl, qq.astype(np.float32)), boxes=[s.box])
    rp.set_state(q, np.zeros_like(q))
    est = rp.estimators()[0]
    V = float(np.prod(s.box))
    lhs = est["P_cv"] * V - n * KB * s.temperature
    beads = q.reshape(P, n, 3)
    qbar = beads.mean(axis=0)
    lists = [neighbors.brute_force_fp32(beads[k].astype(np.float32), s.box, wl.model.cutoff) for k in range(P)]

    def f(e):
        tot = 0.0
        for k in range(P):
            qk = (1.0 + e) * qbar + (beads[k] - qbar)
            G = bpnn.descriptors(wl.model, qk, s.species, s.box * (1.0 + e), np.arange(n), *lists[k])
            tot += bpnn.mlp_energy_grad(wl.model, s.species, bpnn.normalise(wl.model, G, s.species))[0].sum()
        return tot / P
    h = 1e-6
    rhs = -(f(h) - f(-h)) / (2 * h) / 3.0
    assert lhs == pytest.approx(rhs, rel=1e-6, abs=1e-9)


# ---------------------------------------------------------------- QHO closed forms

def test_qho_bead_sum_equals_closed_form_and_limits():
    g = json.load(open(os.path.join(GOLDEN, "qho_s1.json")))
    m, w, T = g["mass_amu"], g["omega_per_fs"], g["temperature_K"]
    beta = 1.0 / (KB * T)
    assert beta * HBAR * w == pytest.approx(g["beta_hbar_omega"], abs=0.01)
    for P in g["beads_sweep"]:
        assert qho.x2_beads_sum(m, w, T, P) == pytest.approx(qho.x2_beads_closed(m, w, T, P), rel=1e-12)
    assert qho.x2_beads_sum(m, w, T, 1) == pytest.approx(qho.x2_classical(m, w, T), rel=1e-14)
    assert qho.x2_beads_sum(m, w, T, 4096) == pytest.approx(qho.x2_exact(m, w, T), rel=1e-6)
    # <E> = k <x^2> reaches hbar w/2 coth(beta hbar w/2) and k_B T in the two limits
    assert qho.energy_beads(m, w, T, 4096) == pytest.approx(qho.energy_exact(w, T), rel=1e-6)
    assert qho.energy_beads(m, w, 5000.0, 1) == pytest.approx(KB * 5000.0, rel=1e-12)
    # the bead sum increases monotonically towards the quantum value
    vals = [qho.x2_beads_sum(m, w, T, P) for P in g["beads_sweep"]]
    assert all(a < b for a, b in zip(vals[:-1], vals[1:]))


# ---------------------------------------------------------------- Sec. S1 protocol, exact
# The three sweeps of Sec. S1 (beads at 10 K, temperature at P = 128, time
# step at 10 K and P = 128) on the stationary covariance of the oracle's own
# step (ring_linear.py): no sampling error, so the finite-P value is checked
# to the integrator's O(dt^2) splitting error.  The text shows the sweeps as
# figures without their abscissae; the temperatures and time steps below are
# a reading.

S1_TEMPERATURES_K = [10.0, 30.0, 100.0, 300.0, 1000.0]
S1_TIME_STEPS_FS = [0.25, 0.5, 1.0, 2.0]


def _oracle_qho_point(P, T, dt, m, w, tau0=100.0):
    """(<x^2> per bead, <K_prim>, <K_cv>) per atom, exact stationary means."""
    steppers = [(2 * P, P, T, np.full(2 * P, m))]

    def one_step(q, p, xi):
        rp = ring.RingPolymers(steppers, dt, tau0, 1.0, 1, ring.harmonic_force_fn(steppers, w))
        rp.set_state(q, p)
        rp.step(noise=xi)
        return rp.q, rp.p
    A, B = ring_linear.step_maps(one_step, P)
    S = ring_linear.stationary_covariance(A, B)
    single = [(1, P, T, np.array([m]))]
    rp = ring.RingPolymers(single, dt, tau0, 1.0, 1, ring.harmonic_force_fn(single, w))

    def estimate(key):
        def f(q):
            rp.set_state(q, np.zeros_like(q))
            return rp.estimators()[0][key]
        return f
    return (ring_linear.bead_x2(S, P), ring_linear.quadratic_mean(estimate("K_prim"), S, P),
            ring_linear.quadratic_mean(estimate("K_cv"), S, P))


def _s1_check(P, T, dt, x2_tol, kprim_tol):
    g = json.load(open(os.path.join(GOLDEN, "qho_s1.json")))
    m, w = g["mass_amu"], g["omega_per_fs"]
    x2, kprim, kcv = _oracle_qho_point(P, T, dt, m, w)
    want = qho.x2_beads_sum(m, w, T, P)
    want_k = 1.5 * qho.energy_beads(m, w, T, P)       # three dimensions, <K> = <V> = E/2 each
    assert x2 == pytest.approx(want, rel=x2_tol)
    assert kcv == pytest.approx(want_k, rel=x2_tol)
    assert kprim == pytest.approx(want_k, rel=kprim_tol)
    return x2, kprim, kcv


@pytest.mark.parametrize("P", json.load(open(os.path.join(GOLDEN, "qho_s1.json")))["beads_sweep"])
def test_s1_bead_sweep_stationary_average_is_the_exact_finite_P_value(P):
    # T = 10 K, dt = 0.5 fs: the splitting error is (w dt)^2 / 4 ~ 1e-5 in <x^2>;
    # K_prim differences the large spring energy and carries it P-fold
    _s1_check(P, 10.0, 0.5, 2e-5, 5e-4)


def test_s1_bead_sweep_converges_to_the_quantum_value():
    g = json.load(open(os.path.join(GOLDEN, "qho_s1.json")))
    m, w, T = g["mass_amu"], g["omega_per_fs"], g["temperature_K"]
    vals = [_oracle_qho_point(P, T, g["dt_fs"], m, w)[0] for P in g["beads_sweep"]]
    assert all(a < b for a, b in zip(vals[:-1], vals[1:]))
    assert vals[0] == pytest.approx(qho.x2_classical(m, w, T), rel=2e-5)
    # 128 beads reach the quantum value to 0.07 % at beta hbar w = 9.5
    assert vals[-1] == pytest.approx(qho.x2_exact(m, w, T), rel=1e-3)


@pytest.mark.parametrize("T", S1_TEMPERATURES_K)
def test_s1_temperature_sweep_at_128_beads(T):
    g = json.load(open(os.path.join(GOLDEN, "qho_s1.json")))
    m, w = g["mass_amu"], g["omega_per_fs"]
    x2, _, kcv = _s1_check(128, T, g["dt_fs"], 2e-5, 3e-3)
    assert x2 == pytest.approx(qho.x2_exact(m, w, T), rel=1e-3)
    assert kcv == pytest.approx(1.5 * qho.energy_exact(w, T), rel=1e-3)


def test_s1_time_step_sweep_converges_as_dt_squared():
    g = json.load(open(os.path.join(GOLDEN, "qho_s1.json")))
    m, w, T = g["mass_amu"], g["omega_per_fs"], g["temperature_K"]
    want = qho.x2_beads_sum(m, w, T, 128)
    want_k = 1.5 * qho.energy_beads(m, w, T, 128)
    ex, ek = [], []
    for dt in S1_TIME_STEPS_FS:
        x2, kprim, _ = _oracle_qho_point(128, T, dt, m, w)
        ex.append(x2 / want - 1.0)
        ek.append(kprim / want_k - 1.0)
    for e in (ex, ek):
        r = np.array(e[1:]) / np.array(e[:-1])
        assert np.all((3.6 < r) & (r < 4.4)), r
    assert abs(ex[0]) < 5e-6 and abs(ek[0]) < 2e-4


# ---------------------------------------------------------------- Philox noise

def test_philox_words_are_uniform_and_counter_sensitive():
    x = np.concatenate(philox.noise_words(4001, 7, 0, 200000))
    u = (x.astype(np.float64) + 0.5) / 2.0 ** 32
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(u))
    counts = np.bincount((x >> np.uint64(24)).astype(np.int64), minlength=256)
    chi2 = np.sum((counts - len(x) / 256) ** 2 / (len(x) / 256))
    assert chi2 < 255 + 5 * np.sqrt(2 * 255)
    a = np.stack(philox.noise_words(4001, 7, 0, 1000))
    for other in (philox.noise_words(4001, 8, 0, 1000), philox.noise_words(4001, 7, 1, 1000),
                  philox.noise_words(4002, 7, 0, 1000)):
        assert np.mean(np.stack(other) == a) < 1e-3
    # a counter in the high step word changes the stream as well
    b = np.stack(philox.noise_words(4001, 7 + (1 << 32), 0, 1000))
    assert np.mean(b == a) < 1e-3


def test_philox_normals_moments():
    z = philox.thermostat_noise(99, 3, 1, 400000).ravel()
    n = len(z)
    assert abs(z.mean()) < 4 / np.sqrt(n)
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / n)
    assert abs(np.mean(z ** 4) - 3) < 4 * np.sqrt(96 / n)
    # the three components are uncorrelated
    zz = philox.thermostat_noise(99, 3, 1, 200000)
    c = np.corrcoef(zz.T)
    assert np.abs(c - np.eye(3)).max() < 4 / np.sqrt(200000)


# ---------------------------------------------------------------- staging (Sec. 2.1)

@pytest.mark.parametrize("P", [2, 4, 8, 32])
def test_staging_transform_round_trip_and_spring_identity(P):
    rng = np.random.default_rng(P)
    r = rng.normal(size=(P, 7, 3))
    u = ring.staging_forward(r)
    assert np.max(np.abs(ring.staging_inverse(u) - r)) < 1e-13
    assert np.array_equal(u[0], r[0])
    # the ring's springs, sum_l |r_{l+1} - r_l|^2, are diagonal in u with weights l/(l-1)
    springs = np.sum((np.roll(r, -1, axis=0) - r) ** 2)
    fac = ring.staging_mass_factors(P)
    assert np.sum(fac[1:, None, None] * u[1:] ** 2) == pytest.approx(springs, rel=1e-12)
    assert fac[0] == 1.0 and fac[1] == 2.0 and fac[-1] == pytest.approx(P / (P - 1))


@pytest.mark.parametrize("P", [2, 4, 8])
def test_staging_forces_are_the_chain_rule_by_central_differences(P):
    rng = np.random.default_rng(10 + P)
    a = rng.normal(size=(P, 3))
    b = rng.normal(size=(P, 3))

    def U(r):                        # a smooth potential of every bead coordinate
        return float(np.sum(a * np.sin(b * r)) + 0.3 * np.sum(r ** 2) * np.sum(np.cos(r)))

    def F(r):
        return -(a * b * np.cos(b * r) + 0.6 * r * np.sum(np.cos(r)) - 0.3 * np.sum(r ** 2) * np.sin(r))
    r = rng.normal(size=(P, 3))
    u = ring.staging_forward(r)
    G = ring.staging_forces(F(r))
    h = 1e-6
    G_fd = np.zeros_like(u)
    for k in range(P):
        for c in range(3):
            up, um = u.copy(), u.copy()
            up[k, c] += h
            um[k, c] -= h
            G_fd[k, c] = -(U(ring.staging_inverse(up)) - U(ring.staging_inverse(um))) / (2 * h)
    assert np.max(np.abs(G - G_fd)) < 1e-7


def test_staging_free_ring_polymer_conserves_energy():
    P, n, T = 8, 5, 300.0
    systems = _systems(n, P, T)
    rp = ring.StagingRingPolymers(systems, 0.5, 0.0, 1.0, 3,
                                  lambda q: (np.zeros(P), np.zeros_like(q)))
    rng = np.random.default_rng(3)
    rp.set_state(rng.normal(0, 0.2, (n * P, 3)), rng.normal(0, 0.3, (n * P, 3)))
    H0 = _hamiltonian(rp, 0.0)
    for _ in range(200):
        rp.step()
    assert _hamiltonian(rp, 0.0) == pytest.approx(H0, rel=1e-11)


@pytest.mark.parametrize("P", [4, 8])
def test_staging_samples_exact_finite_P_harmonic_average(P):
    g = json.load(open(os.path.join(GOLDEN, "qho_s1.json")))
    m, w = g["mass_amu"], g["omega_per_fs"]
    T = 100.0
    n = 600
    systems = _systems(n, P, T, mass=m)
    rp = ring.StagingRingPolymers(systems, g["dt_fs"], 100.0, 1.0, 19, ring.harmonic_force_fn(systems, w))
    rng = np.random.default_rng(9)
    rp.set_state(rng.normal(0, 0.3, (n * P, 3)), rng.normal(0, 0.2, (n * P, 3)))
    for _ in range(1500):
        rp.step()
    x2, kcv, tb = [], [], []
    for t in range(3000):
        rp.step()
        if t % 5 == 0:
            x2.append(np.mean(rp.q ** 2))
            est = rp.estimators()[0]
            kcv.append(est["K_cv"] / (3 * n))
            tb.append(est["T_beads"])
    mean, err = _block_mean(x2)
    want = qho.x2_beads_sum(m, w, T, P)
    assert abs(mean - want) < 3.5 * err + 2e-3 * want
    kmean, kerr = _block_mean(kcv)
    assert abs(kmean - 0.5 * qho.energy_beads(m, w, T, P)) < 3.5 * kerr + 2e-3 * kmean
    tmean, terr = _block_mean(tb)                      # fictitious kinetic masses: still P T
    assert abs(tmean - P * T) < 3.5 * terr + 5e-3 * P * T


# ---------------------------------------------------------------- primitive (Sec. 2.3)

def test_spring_forces_are_minus_the_gradient_of_the_spring_energy():
    rng = np.random.default_rng(40)
    P, n = 6, 3
    m = np.array([1.0, 2.0, 16.0])
    wP = 0.7
    q = rng.normal(size=(P, n, 3))

    def E(x):
        return 0.5 * MVV2E * wP * wP * np.sum(m[None, :, None] * (np.roll(x, -1, axis=0) - x) ** 2)
    F = ring.spring_forces(q, m, wP)
    h = 1e-6
    for (k, i, c) in [(0, 0, 0), (3, 2, 1), (5, 1, 2)]:
        qp, qm = q.copy(), q.copy()
        qp[k, i, c] += h
        qm[k, i, c] -= h
        assert F[k, i, c] == pytest.approx(-(E(qp) - E(qm)) / (2 * h), rel=1e-7)


def test_primitive_single_bead_equals_normal_modes():
    n, T = 20, 300.0
    systems = _systems(n, 1, T)
    fn = ring.harmonic_force_fn(systems, 0.02)
    rng = np.random.default_rng(41)
    q0, p0 = rng.normal(0, 0.2, (n, 3)), rng.normal(0, 0.3, (n, 3))
    a = ring.RingPolymers(systems, 0.5, 50.0, 1.0, 5, fn)
    b = ring.PrimitiveRingPolymers(systems, 0.5, 50.0, 1.0, 5, fn)
    a.set_state(q0, p0)
    b.set_state(q0, p0)
    for _ in range(20):
        a.step()
        b.step()
    assert np.max(np.abs(a.q - b.q)) < 1e-12 and np.max(np.abs(a.p - b.p)) < 1e-12


def test_primitive_nve_error_scales_as_dt_squared():
    # velocity Verlet on the full ring Hamiltonian: energy error ~ dt^2
    P, n, T = 8, 4, 300.0
    systems = _systems(n, P, T)
    fn = ring.harmonic_force_fn(systems, 0.02)
    rng = np.random.default_rng(42)
    q0, p0 = rng.normal(0, 0.05, (n * P, 3)), rng.normal(0, 0.3, (n * P, 3))
    errs = []
    for dt in (0.1, 0.05):
        rp = ring.PrimitiveRingPolymers(systems, dt, 0.0, 1.0, 3, fn)
        rp.set_state(q0, p0)
        H0 = _hamiltonian(rp, rp.E.sum())
        dev = 0.0
        for _ in range(int(round(20.0 / dt))):
            rp.step()
            dev = max(dev, abs(_hamiltonian(rp, rp.E.sum()) - H0))
        errs.append(dev)
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.15)


def test_primitive_samples_exact_finite_P_harmonic_average():
    g = json.load(open(os.path.join(GOLDEN, "qho_s1.json")))
    m, w = g["mass_amu"], g["omega_per_fs"]
    T, P, n = 100.0, 4, 600
    systems = _systems(n, P, T, mass=m)
    # w_P = 0.052/fs at P = 4, T = 100 K: dt = 0.25 fs keeps 2 w_P dt = 0.026
    rp = ring.PrimitiveRingPolymers(systems, 0.25, 50.0, 1.0, 21, ring.harmonic_force_fn(systems, w))
    rng = np.random.default_rng(11)
    rp.set_state(rng.normal(0, 0.3, (n * P, 3)), rng.normal(0, 0.2, (n * P, 3)))
    for _ in range(3000):
        rp.step()
    x2 = []
    for t in range(6000):
        rp.step()
        if t % 10 == 0:
            x2.append(np.mean(rp.q ** 2))
    mean, err = _block_mean(x2)
    want = qho.x2_beads_sum(m, w, T, P)
    # velocity Verlet samples the harmonic ring with an O((w dt)^2) bias, ~1e-4 here
    assert abs(mean - want) < 3.5 * err + 2e-3 * want
