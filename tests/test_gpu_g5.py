"""GPU parity of the G5 angular functions (spherical-harmonic moments, O(K)
per atom) against the FP64 oracle's pair double sum, through the C ABI.

Bars as for the G4 path: descriptors within 1e-5 relative, FP32 path per-atom
force error <= 1e-5 and bead energy error <= 1e-6 (metrics.py), BF16-split
MLP forces <= 2e-2; at the 393 216 bead-atom workload, sampled atoms computed
one by one by the oracle; every launch shape bitwise identical.
"""
import sys

import numpy as np
import pytest

from paper_2503_23728_amd import synthetic as S
from oracle import bpnn, ring
from metrics import energy_error, force_error, rel_max

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_FORCE_TOL = 1e-5
FP32_ENERGY_TOL = 1e-6
BF16_FORCE_TOL = 2e-2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _engine(wl, **kw):
    from paper_2503_23728_amd.pimd import Pimd
    return Pimd.from_workload(wl, device="cuda:0", **kw)


WORKLOADS = {
    "fad-P4": lambda: S.with_g5(S.small_workload("fad", n_beads=4)),
    "water8-P4": lambda: S.with_g5(S.small_workload("water8", n_beads=4)),
    "water64-P32": lambda: S.with_g5(S.workload(2)),
}


def _q(wl, seed):
    return S.perturbed_beads(wl, 0.05, seed=seed)


def _oracle_beads(wl, q32):
    E, F, W, A = [], [], [], []
    off = 0
    for s in wl.systems:
        for _ in range(s.n_beads):
            e, f, w, parts = bpnn.bead_energy_forces(wl.model, q32[off:off + s.n_atoms], s.species, s.box,
                                                     return_parts=True)
            E.append(e)
            F.append(f)
            W.append(w)
            A.append(np.abs(parts["Ei"]).sum())
            off += s.n_atoms
    return np.array(E), np.concatenate(F), np.array(W), np.array(A)


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_g5_descriptors_match_oracle(name):
    wl = WORKLOADS[name]()
    say(f"g5 descriptors {name}")
    eng = _engine(wl)
    q = _q(wl, seed=3)
    eng.energy_forces(torch.from_numpy(q).cuda(), forces=False)
    x = eng.debug_descriptors().cpu().numpy()
    worst, off = 0.0, 0
    for s in wl.systems:
        for _ in range(s.n_beads):
            ref = bpnn.bead_energy_forces(wl.model, q[off:off + s.n_atoms], s.species, s.box,
                                          return_parts=True)[3]["xhat"]
            worst = max(worst, np.max(np.abs(x[off:off + s.n_atoms] - ref) / np.maximum(np.abs(ref), 1e-2)))
            off += s.n_atoms
    say(f"  descriptor rel err {worst:.2e}")
    assert worst < 1e-5


@pytest.mark.parametrize("prec", ["fp64-mlp", "bf16"])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_g5_energy_forces_virial(name, prec):
    wl = WORKLOADS[name]()
    say(f"g5 {prec} forces {name}")
    eng = _engine(wl, precision=prec)
    q = _q(wl, seed=5)
    E, F, W = eng.energy_forces(torch.from_numpy(q).cuda(), forces=True, virial=True)
    E, F, W = E.cpu().numpy(), F.cpu().numpy(), W.cpu().numpy()
    E_ref, F_ref, W_ref, A = _oracle_beads(wl, q)
    fe, ee, we = force_error(F, F_ref), energy_error(E, E_ref, A), rel_max(W, W_ref)
    say(f"  force err {fe:.2e} energy err {ee:.2e} virial err {we:.2e}")
    if prec == "fp64-mlp":
        assert fe < FP32_FORCE_TOL and ee < FP32_ENERGY_TOL and we < 1e-4
    else:
        assert fe < BF16_FORCE_TOL


def test_g5_isolated_atom_and_single_atom_system():
    # an atom with no neighbours has zero moments and zero angular features
    wl = WORKLOADS["fad-P4"]()
    s = wl.systems[0]
    wl.systems = [S.System(s.n_atoms, 2, s.temperature, s.box, s.species, s.q0),
                  S.System(1, 2, 300.0, np.zeros(3), np.array([2], np.int32), np.zeros((1, 3)))]
    say("g5 isolated atom + 1-atom system")
    eng = _engine(wl, precision="fp64-mlp")
    q = _q(wl, seed=4)
    q[3] += np.float32(50.0)
    E, F, _ = eng.energy_forces(torch.from_numpy(q).cuda())
    E_ref, F_ref, _, A = _oracle_beads(wl, q)
    fe = force_error(F.cpu().numpy(), F_ref)
    say(f"  force err {fe:.2e}")
    assert fe < FP32_FORCE_TOL
    assert energy_error(E.cpu().numpy(), E_ref, np.maximum(A, 1e-30)) < FP32_ENERGY_TOL


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_g5_every_launch_shape_gives_bitwise_identical_results(prec):
    wl = WORKLOADS["water64-P32"]()
    say(f"g5 launch shapes {prec}")
    eng = _engine(wl, precision=prec)
    q = torch.from_numpy(_q(wl, seed=9)).cuda()
    E0, F0, W0 = eng.energy_forces(q, virial=True)
    x0 = eng.debug_descriptors()
    for waves in (1, 2, 4):
        for grid in (0, 7, 300):
            fr = (waves + grid) % 2
            eng.set_tuning(centre_waves=waves, centre_grid=grid, force_rows=fr)
            E, F, W = eng.energy_forces(q, virial=True)
            assert torch.equal(E, E0) and torch.equal(F, F0) and torch.equal(W, W0), (waves, grid, fr)
            assert torch.equal(eng.debug_descriptors(), x0), (waves, grid)


def test_g5_one_step_with_injected_noise_matches_oracle():
    wl = WORKLOADS["water8-P4"]()
    say("g5 one step")
    eng = _engine(wl, precision="fp64-mlp")
    q0 = _q(wl, seed=9)
    _, p0 = S.initial_state(wl)
    xi = np.random.default_rng(10).normal(size=(2, len(q0), 3)).astype(np.float32)
    eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda(), step=0)
    eng.inject_noise(torch.from_numpy(xi).cuda())
    eng.step(1)
    q, p, F, step = eng.get_state()
    systems = [(s.n_atoms, s.n_beads, s.temperature, wl.model.masses[s.species]) for s in wl.systems]

    def fn(x):
        E, Fo, _ = bpnn.energy_forces(wl, np.asarray(x, np.float32))
        return E, Fo
    rp = ring.RingPolymers(systems, wl.dt, wl.tau0, wl.pile_lambda, wl.philox_seed, fn)
    rp.set_state(q0.astype(np.float64), p0.astype(np.float64))
    rp.step(noise=xi.astype(np.float64))
    dq = np.max(np.abs(q.cpu().numpy() - rp.q)) / np.max(np.abs(rp.q))
    dp = rel_max(p.cpu().numpy(), rp.p)
    say(f"  dq {dq:.2e} dp {dp:.2e}")
    assert step == 1 and dq < 1e-6 and dp < 1e-5


def test_g5_large_water_sampled_atoms():
    # the full 393 216 bead-atom launch; sampled atoms by the oracle one by one
    wl = S.with_g5(S.workload(5))
    say(f"g5 large water: {wl.bead_atoms} bead-atoms")
    eng = _engine(wl, precision="fp64-mlp")
    q = _q(wl, seed=24)
    E, F, _ = eng.energy_forces(torch.from_numpy(q).cuda())
    F = F.cpu().numpy()
    x = eng.debug_descriptors().cpu().numpy()
    s = wl.systems[0]
    n = s.n_atoms
    rng = np.random.default_rng(25)
    F_rms = np.sqrt(np.mean(np.sum(F[:n] ** 2, axis=1)))
    worst_f, worst_x = 0.0, 0.0
    for bead in (0, 31):
        qb = q[bead * n:(bead + 1) * n]
        atoms = rng.choice(n, 4, replace=False)
        F_ref = bpnn.atom_forces_sampled(wl.model, qb, s.species, s.box, atoms)
        x_ref = bpnn.atom_descriptors_sampled(wl.model, qb, s.species, s.box, atoms)
        got = F[bead * n + atoms]
        e = np.linalg.norm(got - F_ref, axis=1) / np.maximum(np.linalg.norm(F_ref, axis=1), 0.1 * F_rms)
        worst_f = max(worst_f, e.max())
        worst_x = max(worst_x, np.max(np.abs(x[bead * n + atoms] - x_ref) / np.maximum(np.abs(x_ref), 1e-2)))
    say(f"  sampled force err {worst_f:.2e}, descriptor err {worst_x:.2e}")
    assert worst_f < FP32_FORCE_TOL and worst_x < 1e-5
    assert np.all(np.isfinite(E.cpu().numpy()))
