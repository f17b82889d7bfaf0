"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

Bars: neighbour lists bit-exact; FP32 path per-atom force error <= 1e-5 and
bead energy error <= 1e-6 (metrics.py); BF16 MLP path force error <= 2e-2;
one integrator step with injected noise within 1e-6 relative.
"""
import sys

import numpy as np
import pytest

from paper_2503_23728_amd import synthetic as S
from oracle import bpnn, neighbors, philox, ring
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


def _oracle_beads(wl, q32):
    """Per-bead oracle energies, forces, virials and sum_i |E_i|."""
    q32 = np.asarray(q32, np.float32).reshape(-1, 3)
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


WORKLOADS = {
    "fad-P4": lambda: S.small_workload("fad", n_beads=4),
    "water8-P4": lambda: S.small_workload("water8", n_beads=4),
    "water64-P32": lambda: S.workload(2),
    "ice96-P32": lambda: S.workload(3),
}


def _q(wl, seed=1, amp=0.05):
    return S.perturbed_beads(wl, amp, seed=seed)


# ---------------------------------------------------------------- Philox

def test_philox_integer_stream_matches_oracle():
    wl = S.small_workload("fad")
    eng = _engine(wl)
    for step, half in ((0, 0), (7, 1), ((1 << 32) + 3, 0)):
        say(f"philox step={step} half={half}")
        w = eng.debug_philox(step, half, 5000).cpu().numpy().view(np.uint32)
        ref = np.stack(philox.noise_words(wl.philox_seed, step, half, 5000), axis=1).astype(np.uint32)
        assert np.array_equal(w, ref)


# ---------------------------------------------------------------- neighbours

@pytest.mark.parametrize("cells", [0, 1])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_neighbor_lists_bit_exact(name, cells):
    # both periodic search kernels: per centre (0) and per cell with the
    # stencil staged in LDS (1); for molecules without a box, cells = 1 runs
    # the lane-per-centre kernels, which write the lists themselves
    wl = WORKLOADS[name]()
    periodic = any(np.any(np.asarray(s.box) > 0) for s in wl.systems)
    say(f"neighbours {name} cells={cells}")
    eng = _engine(wl)
    if periodic:
        eng.set_tuning(neighbor_cells=cells)
    else:
        eng.set_tuning(centre_lanes=cells)
    q = _q(wl, seed=2, amp=0.3)
    q[::7] += np.float32(25.0)    # unwrapped positions far outside the box
    eng.energy_forces(torch.from_numpy(q).cuda(), forces=False)
    torch.cuda.synchronize()
    off = 0
    bead = 0
    for s in wl.systems:
        for k in range(s.n_beads):
            if k in (0, s.n_beads - 1):
                start, idx = neighbors.brute_force_fp32(q[off:off + s.n_atoms], s.box, wl.model.cutoff)
                ref = np.stack([np.repeat(np.arange(s.n_atoms), np.diff(start)), idx], axis=1)
                got = eng.debug_neighbors(bead)
                assert np.array_equal(got, ref), f"bead {bead}"
            off += s.n_atoms
            bead += 1


def test_neighbor_list_with_isolated_atom_and_single_atom_system():
    wl = S.small_workload("fad", n_beads=2)
    s = wl.systems[0]
    lone = S.System(1, 2, 300.0, np.zeros(3), np.array([2], np.int32), np.zeros((1, 3)))
    wl.systems = [s, lone]
    say("neighbours: isolated atom + 1-atom system")
    eng = _engine(wl)
    q = _q(wl, seed=4)
    q[3] += np.float32(50.0)   # atom 3 of bead 0 far from everything
    E, F, _ = eng.energy_forces(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    got = eng.debug_neighbors(0)
    assert not np.any(got[:, 0] == 3) and not np.any(got[:, 1] == 3)
    assert len(eng.debug_neighbors(2)) == 0
    E_ref, F_ref, _, _ = _oracle_beads(wl, q)
    assert force_error(F.cpu().numpy(), F_ref) < FP32_FORCE_TOL
    assert rel_max(E.cpu().numpy(), E_ref) < 1e-5


# ---------------------------------------------------------------- descriptors

@pytest.mark.parametrize("name", ["fad-P4", "water8-P4", "water64-P32"])
def test_descriptors_match_oracle(name):
    wl = WORKLOADS[name]()
    say(f"descriptors {name}")
    eng = _engine(wl)
    q = _q(wl, seed=3)
    eng.energy_forces(torch.from_numpy(q).cuda(), forces=False)
    x = eng.debug_descriptors().cpu().numpy()
    off = 0
    worst = 0.0
    for s in wl.systems:
        for _ in range(s.n_beads):
            ref = bpnn.bead_energy_forces(wl.model, q[off:off + s.n_atoms], s.species, s.box,
                                          return_parts=True)[3]["xhat"]
            got = x[off:off + s.n_atoms]
            worst = max(worst, np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-2)))
            off += s.n_atoms
    say(f"  descriptor rel err {worst:.2e}")
    # float32 sums of ~1e3 triplet terms, each rounded at ~6e-8 (measured 0.9-2.1e-6)
    assert worst < 5e-6


# ---------------------------------------------------------------- energies and forces

@pytest.mark.parametrize("prec", ["fp64-mlp", "fp32"])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_fp32_energy_forces_virial(name, prec):
    # FP32 descriptors, adjoint and integrator; MLP in FP64 or in FP32 (the
    # plain path: FP32 operands and activations, block-compensated sums)
    wl = WORKLOADS[name]()
    say(f"{prec} forces {name}")
    eng = _engine(wl, precision=prec)
    q = _q(wl, seed=5)
    E, F, W = eng.energy_forces(torch.from_numpy(q).cuda(), forces=True, virial=True)
    E, F, W = E.cpu().numpy(), F.cpu().numpy(), W.cpu().numpy()
    E_ref, F_ref, W_ref, A = _oracle_beads(wl, q)
    fe, ee = force_error(F, F_ref), energy_error(E, E_ref, A)
    we = rel_max(W, W_ref)
    say(f"  force err {fe:.2e} energy err {ee:.2e} virial err {we:.2e}")
    assert fe < FP32_FORCE_TOL
    assert ee < FP32_ENERGY_TOL
    assert we < 1e-4


@pytest.mark.parametrize("chain", [0, 1])
@pytest.mark.parametrize("name", ["water64-P32", "ice96-P32", "fad-P4"])
def test_bf16_mlp_forces(name, chain):
    wl = WORKLOADS[name]()
    say(f"bf16 forces {name} mlp_chain {chain}")
    eng = _engine(wl, precision="bf16")
    eng.set_tuning(mlp_chain=chain)
    q = _q(wl, seed=6)
    E, F, _ = eng.energy_forces(torch.from_numpy(q).cuda())
    E_ref, F_ref, _, A = _oracle_beads(wl, q)
    fe = force_error(F.cpu().numpy(), F_ref)
    say(f"  bf16 (split activations, bfloat16-valued weights) force err {fe:.2e} energy err {energy_error(E.cpu().numpy(), E_ref, A):.2e}")
    assert fe < BF16_FORCE_TOL


FLOAT32_WEIGHTS = {"water64-P32": lambda: S.workload(2, bf16_weights=False),
                   "fad-P4": lambda: S.small_workload("fad", n_beads=4, bf16_weights=False)}


@pytest.mark.parametrize("chain", [0, 1])
@pytest.mark.parametrize("name", list(FLOAT32_WEIGHTS))
def test_bf16_split_with_float32_valued_weights(name, chain):
    # the synthetic weights are bfloat16 values, so the split mode multiplies
    # two activation parts by one weight part; weights with float32 mantissas
    # (a model trained in FP32) make it split the weights too (three products)
    wl = FLOAT32_WEIGHTS[name]()
    assert any(np.any(W.view(np.uint32) & 0xFFFF) for layers in wl.model.weights for W, _ in layers)
    say(f"bf16 split, float32-valued weights {name}, mlp_chain {chain}")
    q = _q(wl, seed=6)
    E_ref, F_ref, _, A = _oracle_beads(wl, q)
    eng = _engine(wl, precision="bf16")
    eng.set_tuning(mlp_chain=chain)
    E, F, _ = eng.energy_forces(torch.from_numpy(q).cuda())
    fe = force_error(F.cpu().numpy(), F_ref)
    ee = energy_error(E.cpu().numpy(), E_ref, A)
    say(f"  force err {fe:.2e} energy err {ee:.2e}")
    assert fe < BF16_FORCE_TOL
    eng.close()


@pytest.mark.parametrize("chain", [0, 1])
@pytest.mark.parametrize("name", ["water64-P32", "fad-P4"])
def test_bf16_plain_mlp_matches_its_emulation(name, chain):
    # one-term BF16 operands: compared with the oracle's BF16-operand emulation
    # (which carries the same roundings), and its error against FP64 reported
    wl = WORKLOADS[name]()
    say(f"bf16-plain forces {name} mlp_chain {chain}")
    eng = _engine(wl, precision="bf16-plain")
    eng.set_tuning(mlp_chain=chain)
    q = _q(wl, seed=6)
    _, F, _ = eng.energy_forces(torch.from_numpy(q).cuda())
    F = F.cpu().numpy()
    _, F_emul, _ = bpnn.energy_forces(wl, q, bf16=True)
    _, F_ref, _ = bpnn.energy_forces(wl, q)
    fe_emul, fe_ref = force_error(F, F_emul), force_error(F, F_ref)
    fe_emul_ref = force_error(F_emul, F_ref)
    say(f"  bf16-plain vs emulation {fe_emul:.2e}, vs FP64 {fe_ref:.2e} (emulation vs FP64 {fe_emul_ref:.2e})")
    # bfloat16 roundings near ties flip between FP32 and FP64 intermediates, so the
    # two agree in the size of their error, not element by element
    assert fe_ref < 2.0 * fe_emul_ref + 1e-3


def test_work_counts_match_oracle():
    wl = WORKLOADS["water64-P32"]()
    say("work counts")
    eng = _engine(wl)
    q = _q(wl, seed=12)
    eng.energy_forces(torch.from_numpy(q).cuda(), forces=False)
    pairs, trip, trip_in = eng.work_counts()
    s = wl.systems[0]
    rp, rt, rti = 0, 0, 0
    for k in range(s.n_beads):
        qb = q[k * s.n_atoms:(k + 1) * s.n_atoms]
        start, idx = neighbors.brute_force_fp32(qb, s.box, wl.model.cutoff)
        _, counts = bpnn.descriptors(wl.model, qb.astype(np.float64), s.species, s.box, np.arange(s.n_atoms),
                                     start, idx, with_counts=True)
        rp += len(idx)
        rt += counts[:, 0].sum()
        rti += counts[:, 1].sum()
    say(f"  pairs {pairs} triplets {trip} in range {trip_in}")
    assert pairs == rp and trip == rt
    assert abs(trip_in - rti) <= 1e-5 * rti


def test_stage_profile_and_eager_steps_match_graph_steps():
    wl = WORKLOADS["water8-P4"]()
    say("stage profile / eager vs graph")
    q0, p0 = S.initial_state(wl)
    a, b = _engine(wl), _engine(wl)
    for e in (a, b):
        e.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    b.set_graph(False)
    a.step(3)
    b.step(3)
    qa, pa, _, sa = a.get_state()
    qb, pb, _, sb = b.get_state()
    assert sa == sb == 3 and torch.equal(qa, qb) and torch.equal(pa, pb)
    ms = a.profile_stages(2)
    assert set(ms) == {"integrate_pre", "neighbors", "descriptors", "mlp", "adjoint", "forces", "integrate_post"}
    assert all(v >= 0 for v in ms.values())
    assert a.get_state()[3] == 5
    # gap-free kernel timing leaves the state and the forces of the positions alone
    q5, p5, F5, _ = a.get_state()
    kt = a.time_stages(3)
    assert set(kt) == {"neighbors", "descriptors", "mlp", "adjoint", "forces"} and all(v > 0 for v in kt.values())
    q6, p6, F6, s6 = a.get_state()
    assert s6 == 5 and torch.equal(q5, q6) and torch.equal(p5, p6) and torch.equal(F5, F6)


def test_forces_are_bitwise_deterministic():
    wl = WORKLOADS["water64-P32"]()
    say("determinism")
    eng = _engine(wl)
    q = torch.from_numpy(_q(wl, seed=7)).cuda()
    _, F1, W1 = eng.energy_forces(q, virial=True)
    _, F2, W2 = eng.energy_forces(q, virial=True)
    assert torch.equal(F1, F2) and torch.equal(W1, W2)


def test_autograd_function_backward_is_minus_forces():
    from paper_2503_23728_amd.pimd import PimdEnergy
    wl = WORKLOADS["water8-P4"]()
    say("autograd")
    eng = _engine(wl)
    q = torch.from_numpy(_q(wl, seed=8)).cuda().requires_grad_(True)
    E = PimdEnergy.apply(q, eng)
    w = torch.linspace(0.5, 1.5, E.numel(), device=E.device)
    (w * E).sum().backward()
    _, F, _ = eng.energy_forces(q.detach())
    rows = eng.bead_of_row
    assert torch.allclose(q.grad, -w[rows][:, None] * F)


# ---------------------------------------------------------------- integrator

def _oracle_rp(wl, q0, p0, force_bf16=False):
    systems = [(s.n_atoms, s.n_beads, s.temperature, wl.model.masses[s.species]) for s in wl.systems]

    def fn(q):
        E, F, _ = bpnn.energy_forces(wl, np.asarray(q, np.float32), bf16=force_bf16)
        return E, F
    rp = ring.RingPolymers(systems, wl.dt, wl.tau0, wl.pile_lambda, wl.philox_seed, fn)
    rp.set_state(q0.astype(np.float64), p0.astype(np.float64))
    return rp


@pytest.mark.parametrize("name", ["fad-P4", "water8-P4"])
def test_one_step_with_injected_noise_matches_oracle(name):
    wl = WORKLOADS[name]()
    say(f"one step {name}")
    eng = _engine(wl)
    q0 = _q(wl, seed=9)
    _, p0 = S.initial_state(wl)
    xi = np.random.default_rng(10).normal(size=(2, len(q0), 3)).astype(np.float32)
    eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda(), step=0)
    eng.inject_noise(torch.from_numpy(xi).cuda())
    eng.step(1)
    q, p, F, step = eng.get_state()
    rp = _oracle_rp(wl, q0, p0)
    rp.step(noise=xi.astype(np.float64))
    dq = np.max(np.abs(q.cpu().numpy() - rp.q)) / np.max(np.abs(rp.q))
    dp = rel_max(p.cpu().numpy(), rp.p)
    say(f"  dq {dq:.2e} dp {dp:.2e}")
    assert step == 1
    assert dq < 1e-6 and dp < 1e-6
    # the forces carried to the next step are those of the GPU's new positions
    _, F_ref, _ = bpnn.energy_forces(wl, q.cpu().numpy())
    assert force_error(F.cpu().numpy(), F_ref) < FP32_FORCE_TOL


def test_graph_steps_follow_oracle_with_philox_noise():
    wl = WORKLOADS["fad-P4"]()
    say("graph steps with Philox noise")
    eng = _engine(wl)
    q0, p0 = S.initial_state(wl)
    eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda(), step=0)
    rp = _oracle_rp(wl, q0, p0)
    for n in range(5):
        eng.step(1)
        rp.step()
    q, p, _, step = eng.get_state()
    assert step == 5
    assert np.max(np.abs(q.cpu().numpy() - rp.q)) < 1e-5
    assert rel_max(p.cpu().numpy(), rp.p) < 1e-4
    est, ref = eng.estimators()[0], rp.estimators()[0]
    for k in ("V_bar", "K_prim", "K_cv", "E_spring", "K_beads", "T_beads", "H_conserved", "heat_bath"):
        assert est[k] == pytest.approx(ref[k], rel=1e-4, abs=1e-5), k


# ---------------------------------------------------------------- failure handling

def test_neighbor_overflow_is_reported():
    wl = WORKLOADS["water64-P32"]()
    say("overflow")
    eng = _engine(wl, max_neighbors=32, regrow=False)
    q0, p0 = S.initial_state(wl)
    eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    from paper_2503_23728_amd.abi import PimdError, PIMD_E_CAPACITY
    with pytest.raises(PimdError) as e:
        eng.estimators()
    assert e.value.status == PIMD_E_CAPACITY


def test_nonfinite_state_is_reported():
    wl = WORKLOADS["fad-P4"]()
    say("non-finite")
    eng = _engine(wl)
    q0, p0 = S.initial_state(wl)
    p0 = p0.copy()
    p0[3, 1] = np.nan
    eng.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    from paper_2503_23728_amd.abi import PimdError, PIMD_E_NONFINITE
    with pytest.raises(PimdError) as e:
        eng.get_state()
    assert e.value.status == PIMD_E_NONFINITE


def test_step_before_state_is_an_order_error():
    wl = WORKLOADS["fad-P4"]()
    eng = _engine(wl)
    from paper_2503_23728_amd.abi import PimdError, PIMD_E_STATE
    with pytest.raises(PimdError) as e:
        eng.step(1)
    assert e.value.status == PIMD_E_STATE


# ---------------------------------------------------------------- launch shapes / autotuner

@pytest.mark.parametrize("name", ["water64-P32", "fad-P4"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_every_launch_shape_gives_bitwise_identical_results(name, prec):
    wl = WORKLOADS[name]()
    say(f"launch shapes {name} {prec}")
    eng = _engine(wl, precision=prec)
    q = torch.from_numpy(_q(wl, seed=9)).cuda()
    # every shape within each kernel family: lane or wave per centre (molecules
    # without a box), and the register-chained or LDS-staged BF16 MLP; the
    # families agree to rounding
    lanes_modes = (1, 0) if eng.get_tuning()["centre_lanes"] else (0,)
    chain_modes = (0, 1) if prec == "bf16" else (0,)
    first = None
    for lanes, chain in [(a, b) for a in lanes_modes for b in chain_modes]:
        eng.set_tuning(centre_lanes=lanes, mlp_chain=chain, centre_waves=4, centre_grid=0, mlp_rows=32)
        E0, F0, W0 = eng.energy_forces(q, virial=True)
        x0 = eng.debug_descriptors()
        if first is None:
            first = (E0, F0, x0)
        else:
            # FP32: the energy bar; the BF16 split holds 16 significant bits of
            # each activation (hi + lo), so a one-ulp change of a descriptor can
            # move an activation's representation by up to 2^-17 of it
            e_tol = 1e-6 if prec == "fp32" else 2.0 ** -16
            assert rel_max(F0.cpu().numpy(), first[1].cpu().numpy()) < 1e-5
            assert rel_max(E0.cpu().numpy(), first[0].cpu().numpy()) < e_tol
            assert rel_max(x0.cpu().numpy(), first[2].cpu().numpy()) < 1e-5
        for waves in (1, 2, 4):
            for grid in (0, 7, 300):
                for rows in (16, 32, 64):
                    cells = (waves + rows // 16) % 2
                    mw = 8 if (grid + rows) % 3 else 4
                    fr = (waves + grid + rows // 16) % 2
                    eng.set_tuning(centre_waves=waves, centre_grid=grid, mlp_rows=rows, neighbor_cells=cells,
                                   mlp_waves=mw, force_rows=fr)
                    E, F, W = eng.energy_forces(q, virial=True)
                    shape = (lanes, chain, waves, grid, rows, cells, mw, fr)
                    assert torch.equal(E, E0) and torch.equal(F, F0) and torch.equal(W, W0), shape
                    assert torch.equal(eng.debug_descriptors(), x0), shape


def test_autotune_picks_a_valid_shape_and_the_cache_reapplies_it(tmp_path, monkeypatch):
    from paper_2503_23728_amd import tuning
    monkeypatch.setenv("PIMD_TUNING_CACHE", str(tmp_path / "tuning.json"))
    wl = WORKLOADS["water64-P32"]()
    say("autotune")
    q0, p0 = S.initial_state(wl)
    a = _engine(wl, precision="bf16")
    a.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    _, _, F_before, step0 = a.get_state()
    chain0 = a.get_tuning()["mlp_chain"]
    shape, cached = a.autotune(n_reps=2)
    assert not cached
    assert shape["centre_waves"] in (1, 2, 4) and shape["mlp_rows"] in (16, 32, 64) and shape["centre_grid"] >= 0
    assert shape["neighbor_cells"] in (0, 1) and shape["mlp_waves"] in (4, 8) and shape["force_rows"] in (0, 1)
    # the state does not move and the forces are those of the same positions
    # (bitwise within a kernel family; the chained and LDS-staged MLPs sum in
    # another order)
    _, _, F_after, step1 = a.get_state()
    assert step1 == step0
    if shape["mlp_chain"] == chain0:
        assert torch.equal(F_before, F_after)
    else:
        assert rel_max(F_after.cpu().numpy(), F_before.cpu().numpy()) < 1e-5
    assert tuning.load(a.tuning_key()) == shape
    b = _engine(wl, precision="bf16")
    b.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda())
    shape_b, cached_b = b.autotune(n_reps=2)
    assert cached_b and shape_b == shape and b.get_tuning() == shape
    # tuned and untuned contexts step identically
    a.step(3)
    b.set_tuning(centre_waves=4, centre_grid=0, mlp_rows=16)
    b.step(3)
    assert torch.equal(a.get_state()[0], b.get_state()[0])


def test_bad_launch_shapes_are_rejected():
    from paper_2503_23728_amd.abi import PimdError, PIMD_E_ARG, PIMD_E_UNSUPPORTED
    wl = WORKLOADS["fad-P4"]()
    eng = _engine(wl)
    for bad in ({"centre_waves": 3}, {"centre_waves": 8}, {"mlp_rows": 48}, {"centre_grid": -1}, {"neighbor_cells": 2},
                {"mlp_waves": 6}, {"force_rows": 2}, {"centre_lanes": 2}, {"mlp_chain": 2}):
        with pytest.raises(PimdError) as ei:
            eng.set_tuning(**bad)
        assert ei.value.status == PIMD_E_ARG
    water = _engine(WORKLOADS["water8-P4"]())     # a box: wave-per-centre kernels only
    assert water.get_tuning()["centre_lanes"] == 0
    with pytest.raises(PimdError) as ei:
        water.set_tuning(centre_lanes=1)
    assert ei.value.status == PIMD_E_UNSUPPORTED
    f64 = _engine(wl, precision="fp64-mlp")
    with pytest.raises(PimdError) as ei:
        f64.set_tuning(mlp_rows=32)
    assert ei.value.status == PIMD_E_UNSUPPORTED
    for prec in ("fp32", "fp64-mlp"):          # the chained MLP is a BF16 kernel
        with pytest.raises(PimdError) as ei:
            _engine(wl, precision=prec).set_tuning(mlp_chain=1)
        assert ei.value.status == PIMD_E_UNSUPPORTED
    with pytest.raises(PimdError):
        eng.autotune(n_reps=1, cache=False)     # no state yet
