"""GPU parity of PILE-G (a global stochastic-velocity-rescaling thermostat on
every system's centroid, Langevin friction on the other modes) and of the
centroid-virial pressure estimator, against the FP64 oracle.

* one step with injected noise (the centroid factor takes its random numbers
  from the centroid rows of the same noise) on formic acid, water 8 and a
  ragged batch with P = 8 ... 64;
* five steps with Philox noise;
* PILE-G samples the exact finite-P harmonic <x^2> (Sec. S1 oscillator);
* P_cv of periodic systems against the oracle's estimator, and 0 without a box.
"""
import sys

import numpy as np
import pytest

from paper_2503_23728_amd import synthetic as S
from oracle import bpnn, qho, ring
from metrics import rel_max

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _engine(wl, **kw):
    from paper_2503_23728_amd.pimd import Pimd
    return Pimd.from_workload(wl, device="cuda:0", thermostat="pile-g", **kw)


def _oracle(wl, q0, p0):
    systems = [(s.n_atoms, s.n_beads, s.temperature, wl.model.masses[s.species]) for s in wl.systems]
    rp = ring.RingPolymers(systems, wl.dt, wl.tau0, wl.pile_lambda, wl.philox_seed,
                           lambda qq: bpnn.energy_forces(wl, qq.astype(np.float32)), thermostat="pile-g",
                           boxes=[s.box for s in wl.systems])
    rp.set_state(np.asarray(q0, np.float64), np.asarray(p0, np.float64))
    return rp


def _ragged():
    full = S.workload(4)
    pick = []
    for P in (8, 16, 32, 64):
        pick += [s for s in full.systems if s.n_beads == P][:2]
    return S.Workload("ragged", pick, full.model, full.dt, full.tau0, full.pile_lambda, 1, full.philox_seed,
                      full.momentum_seed)


CASES = {"fad-P4": lambda: S.small_workload("fad", n_beads=4),
         "water8-P4": lambda: S.small_workload("water8", n_beads=4),
         "ragged": _ragged}


@pytest.mark.parametrize("name", list(CASES))
def test_pile_g_step_with_injected_noise_matches_oracle(name):
    wl = CASES[name]()
    say(f"PILE-G one step {name}")
    eng = _engine(wl, precision="fp32")
    q0 = S.perturbed_beads(wl, 0.03, seed=51)
    _, p0 = S.initial_state(wl)
    xi = np.random.default_rng(52).normal(size=(2, len(q0), 3)).astype(np.float32)
    eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    eng.inject_noise(torch.from_numpy(xi).cuda())
    eng.step(1)
    q, p, _, step = eng.get_state()
    rp = _oracle(wl, q0, p0)
    rp.step(noise=xi.astype(np.float64))
    dq = np.max(np.abs(q.cpu().numpy() - rp.q)) / np.max(np.abs(rp.q))
    dp = rel_max(p.cpu().numpy(), rp.p)
    say(f"  dq {dq:.2e} dp {dp:.2e}")
    assert step == 1 and dq < 1e-6 and dp < 1e-6
    for a, b in zip(eng.estimators(), rp.estimators()):
        for k in ("K_beads", "heat_bath", "K_cv", "E_spring", "H_conserved", "P_cv"):
            assert a[k] == pytest.approx(b[k], rel=1e-4, abs=1e-7), k


def test_pile_g_philox_steps_follow_oracle():
    wl = CASES["water8-P4"]()
    say("PILE-G Philox steps")
    eng = _engine(wl, precision="fp32")
    q0, p0 = S.initial_state(wl)
    eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    rp = _oracle(wl, q0, p0)
    for _ in range(5):
        eng.step(1)
        rp.step()
    q, p, _, step = eng.get_state()
    assert step == 5
    dq, dp = np.max(np.abs(q.cpu().numpy() - rp.q)), rel_max(p.cpu().numpy(), rp.p)
    say(f"  after 5 steps: |dq| {dq:.2e} A, dp {dp:.2e}")
    assert dq < 1e-5 and dp < 1e-5
    est, ref = eng.estimators()[0], rp.estimators()[0]
    for k in ("K_beads", "heat_bath", "K_cv", "H_conserved", "P_cv"):
        assert est[k] == pytest.approx(ref[k], rel=1e-4, abs=1e-7), k


def test_pile_g_samples_exact_finite_P_harmonic_average():
    from paper_2503_23728_amd.pimd import Pimd
    m, w, T, P, n = 1.008, 0.01244, 100.0, 8, 2048
    say("PILE-G QHO sampling")
    sys_ = S.System(n, P, T, np.zeros(3), np.zeros(n, np.int32), np.zeros((n, 3)))
    eng = Pimd([sys_], None, 0.5, 100.0, 1.0, 61, potential="harmonic", omega=w, masses=np.array([m]),
               device="cuda:0", thermostat="pile-g")
    rng = np.random.default_rng(62)
    eng.set_state(torch.from_numpy(rng.normal(0, 0.3, (n * P, 3)).astype(np.float32)).cuda(),
                  torch.from_numpy(rng.normal(0, 0.2, (n * P, 3)).astype(np.float32)).cuda())
    eng.step(2000)
    x2, kcv = [], []
    for _ in range(200):
        eng.step(20)
        q = eng.get_state(forces=False)[0]
        x2.append(float((q.double() ** 2).mean()))
        kcv.append(eng.estimators()[0]["K_cv"] / (3 * n))
    b = [v.mean() for v in np.array_split(np.array(x2), 20)]
    mean, err = np.mean(b), np.std(b, ddof=1) / np.sqrt(len(b))
    want = qho.x2_beads_sum(m, w, T, P)
    say(f"  <x^2> {mean:.5f} +- {err:.5f}, exact finite-P {want:.5f}")
    assert abs(mean - want) < 4 * err + 3e-3 * want
    want_k = 0.5 * qho.energy_beads(m, w, T, P)
    assert abs(np.mean(kcv) - want_k) < 3e-2 * want_k
    assert eng.estimators()[0]["P_cv"] == 0.0        # no box


@pytest.mark.parametrize("cfg", [2, 3])
def test_centroid_virial_pressure_matches_oracle(cfg):
    from paper_2503_23728_amd.pimd import Pimd
    wl = S.workload(cfg)
    say(f"P_cv workload {cfg}")
    eng = Pimd.from_workload(wl, device="cuda:0", precision="fp32")
    q0 = S.perturbed_beads(wl, 0.05, seed=63)
    _, p0 = S.initial_state(wl)
    eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    got = eng.estimators()[0]
    rp = _oracle(wl, q0, p0)
    ref = rp.estimators()[0]
    say(f"  P_cv {got['P_cv']:.6e} (oracle {ref['P_cv']:.6e}) eV/A^3")
    assert got["P_cv"] == pytest.approx(ref["P_cv"], rel=1e-4)
    # after steps the estimator follows the new state's virial
    eng.step(3)
    q, p, _, _ = eng.get_state(forces=False)
    rp2 = _oracle(wl, q.cpu().numpy(), p.cpu().numpy())
    assert eng.estimators()[0]["P_cv"] == pytest.approx(rp2.estimators()[0]["P_cv"], rel=1e-4)
