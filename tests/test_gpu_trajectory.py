"""Oracle-matching trajectories, read as single-step resynchronisation (MD is
chaotic, so free FP32 and FP64 runs part ways): a GPU trajectory runs with
its own Philox noise, and at every step (formic acid dimer, P = 8, 500 steps)
or every 10th step (water 64 and ice 96, P = 32, 200 steps) its state is
handed to the FP64 oracle and to a second GPU context, both take one step
with the same injected noise, and positions and momenta agree within 1e-6
relative.  The normal-mode PILE-L step of Sec. 2.1 with the thermostat of
Table S3; the FP32 path (FP32 MLP with compensated sums).
"""
import sys

import numpy as np
import pytest

from paper_2503_23728_amd import synthetic as S
from oracle import bpnn, ring

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("cfg,steps,every", [(1, 500, 1), (2, 200, 10), (3, 200, 10)])
def test_single_step_resync_along_a_trajectory(cfg, steps, every):
    from paper_2503_23728_amd.pimd import Pimd
    wl = S.workload(cfg)
    say(f"resync workload {cfg} ({wl.name}): {steps} steps, every {every}")
    traj = Pimd.from_workload(wl, device="cuda:0", precision="fp32")
    one = Pimd.from_workload(wl, device="cuda:0", precision="fp32")
    q0, p0 = S.initial_state(wl)
    traj.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    systems = [(s.n_atoms, s.n_beads, s.temperature, wl.model.masses[s.species]) for s in wl.systems]
    rp = ring.RingPolymers(systems, wl.dt, wl.tau0, wl.pile_lambda, wl.philox_seed,
                           lambda qq: bpnn.energy_forces(wl, qq.astype(np.float32))[:2])
    rng = np.random.default_rng(500 + cfg)
    worst_q = worst_p = 0.0
    for t in range(0, steps, every):
        q, p, _, step = traj.get_state(forces=False)
        assert step == t
        xi = rng.normal(size=(2, len(q0), 3)).astype(np.float32)
        one.set_state(q, p, step=t)
        one.inject_noise(torch.from_numpy(xi).cuda())
        one.step(1)
        q1, p1, _, _ = one.get_state(forces=False)
        rp.set_state(q.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64), step=t)
        rp.step(noise=xi.astype(np.float64))
        dq = np.max(np.abs(q1.cpu().numpy() - rp.q)) / np.max(np.abs(rp.q))
        dp = np.max(np.abs(p1.cpu().numpy() - rp.p)) / np.max(np.abs(rp.p))
        worst_q, worst_p = max(worst_q, dq), max(worst_p, dp)
        assert dq < 1e-6 and dp < 1e-6, (t, dq, dp)
        traj.step(every)
    say(f"  worst one-step error over {steps // every} resyncs: q {worst_q:.2e}, p {worst_p:.2e}")
    assert np.all(np.isfinite(traj.get_state(forces=False)[0].cpu().numpy()))
    traj.close()
    one.close()
