"""GPU: failure handling of the integrator.

A neighbour overflow (an atom with more neighbours than the slots per atom)
latched during a step freezes the state at the last step that completed
without one: later steps enqueued before the fault is read change nothing.
The Python layer then rebuilds the context with more slots, puts the frozen
state back and replays the lost steps.  The input is two water clusters
flying at each other (synthetic.colliding_clusters): every atom starts with
8 neighbours, and the count passes 16 near step 89 (FP64 oracle run), so a
context with 16 slots overflows in the middle of a run.
"""
import sys

import numpy as np
import pytest

from paper_2503_23728_amd import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_STEPS = 120


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _engine(wl, q, p, **kw):
    from paper_2503_23728_amd.pimd import Pimd
    e = Pimd.from_workload(wl, device="cuda:0", precision="fp32", **kw)
    e.set_state(torch.from_numpy(q).cuda(), torch.from_numpy(p).cuda())
    return e


def test_overflow_inside_steps_freezes_the_state_at_the_last_good_step():
    from paper_2503_23728_amd.abi import PimdError, PIMD_E_CAPACITY
    wl, q, p = S.colliding_clusters()
    say("faults: step-by-step reference, 16 slots")
    ref = _engine(wl, q, p, max_neighbors=16, regrow=False)
    last = None
    fail_at = None
    for n in range(1, N_STEPS + 1):
        ref.step(1)
        try:
            ref.check()
        except PimdError as e:
            assert e.status == PIMD_E_CAPACITY
            fail_at = n
            break
        qa, pa, _, sa = ref.get_state(forces=False)
        last = (qa.clone(), pa.clone(), sa, ref.get_heat_bath())
    say(f"faults: first overflow in step {fail_at}")
    assert fail_at is not None and 20 < fail_at < N_STEPS
    # the failing step left the state as it was
    qf, pf, _, sf = ref.get_state(forces=False)
    assert sf == fail_at - 1 == last[2]
    assert torch.equal(qf, last[0]) and torch.equal(pf, last[1])
    say("faults: all steps in one call (graph replays)")
    eng = _engine(wl, q, p, max_neighbors=16, regrow=False)
    eng.step(N_STEPS)
    with pytest.raises(PimdError) as e:
        eng.estimators()
    assert e.value.status == PIMD_E_CAPACITY
    qb, pb, _, sb = eng.get_state(forces=False)
    assert sb == fail_at - 1
    assert torch.equal(qb, last[0]) and torch.equal(pb, last[1])
    assert eng.get_heat_bath() == last[3]


def test_regrow_replays_the_lost_steps():
    wl, q, p = S.colliding_clusters()
    say("faults: regrow from 16 slots")
    eng = _engine(wl, q, p, max_neighbors=16)
    eng.step(N_STEPS)
    est = eng.estimators()[0]
    qa, pa, Fa, sa = eng.get_state()
    assert eng.regrowths == 1 and eng.max_neighbors == 32 and sa == N_STEPS
    say("faults: reference with 32 slots")
    ref = _engine(wl, q, p, max_neighbors=32)
    ref.step(N_STEPS)
    est_ref = ref.estimators()[0]
    qr, pr, Fr, sr = ref.get_state()
    assert ref.regrowths == 0 and sr == N_STEPS
    say(f"faults: regrown run bitwise equal: {torch.equal(qa, qr) and torch.equal(pa, pr)}")
    assert torch.allclose(qa, qr, rtol=0, atol=1e-5)
    assert torch.allclose(pa, pr, rtol=1e-5, atol=1e-6)
    for k in ("V_bar", "K_beads", "H_conserved"):
        assert est[k] == pytest.approx(est_ref[k], rel=1e-5, abs=1e-6), k


def test_energy_forces_reports_and_regrows_an_overflow():
    from paper_2503_23728_amd.abi import PimdError, PIMD_E_CAPACITY
    wl, q, p = S.colliding_clusters()
    # positions where the clusters overlap: free flight of 100 steps
    m = wl.model.masses[wl.systems[0].species]
    qx = q.copy()
    n = wl.systems[0].n_atoms
    for k in range(wl.systems[0].n_beads):
        qx[k * n:(k + 1) * n] += 100 * wl.dt * p[k * n:(k + 1) * n] / m[:, None]
    qt = torch.from_numpy(qx).cuda()
    say("faults: energy_forces at overlapping clusters")
    small = _engine(wl, q, p, max_neighbors=16, regrow=False)
    with pytest.raises(PimdError) as e:
        small.energy_forces(qt)
    assert e.value.status == PIMD_E_CAPACITY
    grown = _engine(wl, q, p, max_neighbors=16)
    E, F, _ = grown.energy_forces(qt)
    big = _engine(wl, q, p, max_neighbors=32)
    Er, Fr, _ = big.energy_forces(qt)
    assert grown.regrowths == 1
    assert torch.equal(E, Er) and torch.equal(F, Fr)


def test_checkpoint_carries_the_heat_bath():
    wl = S.workload(2)
    q0, p0 = S.initial_state(wl)
    say("faults: heat bath through a checkpoint")
    a = _engine(wl, q0, p0, neighbor_skin=2.0)
    a.step(20)
    q, p, _, step = a.get_state()
    saved = (q.clone(), p.clone(), step, a.get_heat_bath())
    assert saved[3][0] != 0.0
    a.step(20)
    est_a = a.estimators()[0]
    b = _engine(wl, q0, p0, neighbor_skin=2.0)
    b.set_state(saved[0], saved[1], step=saved[2], heat_bath=saved[3])
    b.step(20)
    est_b = b.estimators()[0]
    for k, v in est_a.items():
        assert est_b[k] == v, k
