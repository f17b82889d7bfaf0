"""GPU: shared neighbour lists with a skin (one list per atom of the ring-
polymer centroids, rebuilt on demand, filtered per bead each evaluation).

The filtered lists must equal the per-bead lists key for key, so everything
downstream is bitwise the same: lists against the FP32 brute-force oracle,
forces and whole trajectories against the cell-list path of the same engine
settings, with skins that force a rebuild at every step and skins that keep
a list for many steps.
"""
import sys

import numpy as np
import pytest

from paper_2503_23728_amd import synthetic as S
from oracle import neighbors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _engine(wl, **kw):
    from paper_2503_23728_amd.pimd import Pimd
    return Pimd.from_workload(wl, device="cuda:0", **kw)


@pytest.mark.parametrize("name,skin", [("water64", 0.3), ("water64", 3.0), ("ice96", 2.0)])
def test_skin_lists_match_oracle_and_forces_match_cell_lists(name, skin):
    wl = S.workload(2) if name == "water64" else S.workload(3)
    say(f"skin lists {name} skin {skin}")
    ref = _engine(wl, precision="fp32")
    eng = _engine(wl, precision="fp32", neighbor_skin=skin)
    q = S.perturbed_beads(wl, 0.05, seed=3)
    qt = torch.from_numpy(q).cuda()
    E0, F0, W0 = ref.energy_forces(qt, virial=True)
    E1, F1, W1 = eng.energy_forces(qt, virial=True)
    assert torch.equal(E0, E1) and torch.equal(F0, F1) and torch.equal(W0, W1)
    s = wl.systems[0]
    for bead in (0, s.n_beads - 1):
        got = eng.debug_neighbors(bead)
        qb = q[bead * s.n_atoms:(bead + 1) * s.n_atoms]
        start, idx = neighbors.brute_force_fp32(qb, s.box, wl.model.cutoff)
        want = np.stack([np.repeat(np.arange(s.n_atoms), np.diff(start)), idx], axis=1)
        assert np.array_equal(np.asarray(got), want)
    assert eng.neighbor_rebuilds()[0] >= 1


@pytest.mark.parametrize("model", ["g5", "gfn"])
def test_skin_gives_the_same_forces_for_every_model(model):
    # the G5 descriptors and the direct-force head read the same lists
    wl = S.with_g5(S.workload(2)) if model == "g5" else S.gfn_workload(2)
    say(f"skin with the {model} model")
    q = torch.from_numpy(S.perturbed_beads(wl, 0.05, seed=6)).cuda()
    ref = _engine(wl, precision="bf16")
    eng = _engine(wl, precision="bf16", neighbor_skin=2.0)
    _, F0, _ = ref.energy_forces(q)
    _, F1, _ = eng.energy_forces(q)
    assert torch.equal(F0, F1)
    q0, p0 = S.initial_state(wl)
    for e in (ref, eng):
        e.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda(), step=0)
        e.step(10)
    assert torch.equal(ref.get_state()[0], eng.get_state()[0])


def test_skin_ring_wider_than_skin_scans_whole_beads():
    # every 7th bead-atom moved 25 A in unwrapped coordinates (not a box vector):
    # those rings are far wider than the skin, so the step tests every atom
    wl = S.workload(2)
    say("skin: rings wider than the skin")
    eng = _engine(wl, precision="fp32", neighbor_skin=2.0)
    q = S.perturbed_beads(wl, 0.3, seed=2)
    q[::7] += np.float32(25.0)
    eng.energy_forces(torch.from_numpy(q).cuda(), forces=False)
    builds, scans = eng.neighbor_rebuilds()
    assert builds >= 1 and scans >= 1
    s = wl.systems[0]
    for bead in (0, 5, s.n_beads - 1):
        qb = q[bead * s.n_atoms:(bead + 1) * s.n_atoms]
        start, idx = neighbors.brute_force_fp32(qb, s.box, wl.model.cutoff)
        want = np.stack([np.repeat(np.arange(s.n_atoms), np.diff(start)), idx], axis=1)
        assert np.array_equal(np.asarray(eng.debug_neighbors(bead)), want), bead


@pytest.mark.parametrize("skin", [0.3, 3.0])
def test_skin_trajectory_is_bitwise_the_cell_list_trajectory(skin):
    wl = S.workload(2)
    say(f"skin trajectory skin {skin}")
    q0, p0 = S.initial_state(wl)
    out = []
    for kw in ({}, {"neighbor_skin": skin}):
        eng = _engine(wl, precision="bf16", **kw)
        eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda(), step=0)
        eng.step(40)
        q, p, F, step = eng.get_state()
        out.append((q.clone(), p.clone(), F.clone(), step, eng))
    (qa, pa, Fa, sa, _), (qb, pb, Fb, sb, eng) = out
    builds, scans = eng.neighbor_rebuilds()
    say(f"  {builds} builds, {scans} whole-bead scans in 40 steps")
    assert sa == sb == 40
    assert torch.equal(qa, qb) and torch.equal(pa, pb) and torch.equal(Fa, Fb)
    if skin < 1.0:
        # rings spread ~1 A about their centroids: rebuilt at every step, and
        # wider than the skin, so whole beads are scanned
        assert builds > 20 and scans > 20
    else:
        assert builds < 10 and scans == 0


def test_skin_long_trajectory_is_bitwise_the_cell_list_trajectory():
    # 400 steps (100 fs) from the classical geometry: the rings spread to their
    # thermal size and the centroids diffuse, so the lists are rebuilt many times
    wl = S.workload(2)
    say("skin: 400-step trajectory")
    q0, p0 = S.initial_state(wl)
    states = []
    for kw in ({}, {"neighbor_skin": 2.0}):
        eng = _engine(wl, precision="bf16", **kw)
        eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda(), step=0)
        eng.step(400)
        q, p, F, step = eng.get_state()
        states.append((q.clone(), p.clone(), F.clone(), step, eng.estimators()[0]))
    builds, scans = eng.neighbor_rebuilds()
    say(f"  {builds} builds, {scans} whole-bead scans in 400 steps")
    (qa, pa, Fa, sa, ea), (qb, pb, Fb, sb, eb) = states
    assert sa == sb == 400
    assert torch.equal(qa, qb) and torch.equal(pa, pb) and torch.equal(Fa, Fb)
    assert ea == eb
    assert 5 <= builds <= 200 and scans == 0


def test_skin_rebuilds_after_positions_jump():
    wl = S.workload(2)
    say("skin: a jump of the positions forces a rebuild")
    ref = _engine(wl, precision="fp32")
    eng = _engine(wl, precision="fp32", neighbor_skin=3.0)
    q1 = torch.from_numpy(S.perturbed_beads(wl, 0.05, seed=4)).cuda()
    eng.energy_forces(q1)
    n1 = eng.neighbor_rebuilds()[0]
    eng.energy_forces(q1)
    assert eng.neighbor_rebuilds()[0] == n1         # same positions: the lists are kept
    n = wl.systems[0].n_atoms
    q2 = q1.clone().view(-1, n, 3)
    q2[:, :5] += 2.5                                # five whole rings move by 4.3 A
    q2 = q2.view(-1, 3)
    _, F0, _ = ref.energy_forces(q2)
    _, F1, _ = eng.energy_forces(q2)
    assert eng.neighbor_rebuilds() == (n1 + 1, 0)
    assert torch.equal(F0, F1)
    q3 = q2.clone()
    q3[:5] += 2.5                                   # bead 0 only: those rings now exceed the skin
    _, F0, _ = ref.energy_forces(q3)
    _, F1, _ = eng.energy_forces(q3)
    assert eng.neighbor_rebuilds() == (n1 + 2, 1)
    assert torch.equal(F0, F1)


def test_skin_large_water_forces_match_cell_lists():
    wl = S.workload(5)
    say(f"skin: large water, {wl.bead_atoms} bead-atoms")
    q = torch.from_numpy(S.perturbed_beads(wl, 0.05, seed=24)).cuda()
    ref = _engine(wl, precision="bf16")
    _, F0, _ = ref.energy_forces(q)
    F0 = F0.clone()
    del ref
    torch.cuda.empty_cache()
    eng = _engine(wl, precision="bf16", neighbor_skin=2.0)
    _, F1, _ = eng.energy_forces(q)
    assert torch.equal(F0, F1)
    q0, p0 = S.initial_state(wl)
    eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    eng.step(3)
    assert eng.get_state()[3] == 3
