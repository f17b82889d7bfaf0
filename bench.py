"""Throughput of the ML-PIMD hot path on one MI355X.

One step = one full normal-mode PILE-L integrator step of every bead of
every ring polymer: O/B/A in normal modes, neighbour search, descriptors,
MLP, adjoint forces, B/O.  The state is resident in HBM before the timed
region; the timed region is exactly `--steps` steps.

Prints one JSON line: bead-atom force evaluations per second (the whole
job), ns/day, the plain-FP32 comparison path (FP32 MLP, every kernel
enqueued one by one, one context per system), the roofline of the dominant
kernel (algorithmic FLOPs per launch / mean launch time from HIP events on
the launch stream, against the FP32 vector peak) and the FP64 CPU oracle
timed on a bounded sample on the host cores.

Workloads (--config): 1 formic-acid-dimer 10 atoms P=8; 2 water 64 H2O P=32;
3 ice 96 H2O P=32; 4 512 dimer-like ring polymers with P in {8,16,32,64};
5 water 4096 H2O P=32 (default: the largest workload, 393,216 bead-atoms).
The default run also reports, as extra keys, the same workload with every
bead's neighbour list searched through cell lists each step, and the batched
workload 4 against its plain-FP32 path.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
BF16_MFMA_PEAK_TFLOPS = 2500.0      # MI355X published dense BF16 matrix peak
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6      # MI355X published FP64 vector peak
# the adjoint's translation unit and every local header it includes
ADJOINT_SOURCES = ["paper_2503_23728_amd/csrc/k_descriptors.hip", "paper_2503_23728_amd/csrc/device_common.hpp",
                   "paper_2503_23728_amd/csrc/pair_terms.hpp", "paper_2503_23728_amd/csrc/pimd_internal.hpp"]


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"adjoint_traffic_{workload}.json")


def measured_traffic(workload):
    """HBM bytes per k_adjoint launch from the committed rocprofv3 counters, when
    they were taken on this workload and the kernel's sources have not changed
    since (SHA-256 over ADJOINT_SOURCES, in order)."""
    import hashlib
    try:
        rec = json.load(open(traffic_file(workload)))
        if rec["sources"] != ADJOINT_SOURCES:
            return None
        src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in ADJOINT_SOURCES)
    except (OSError, ValueError, KeyError, TypeError):
        return None
    if rec.get("workload") != workload or hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return rec["hbm_read_bytes"] + rec["hbm_write_bytes"]


def mlp_flops_per_row(D, hidden):
    """Multiply-adds of one row: forward through the hidden layers and the
    readout, then the input gradient back through every layer (x2 FLOPs)."""
    sizes = [D] + list(hidden)
    fwd = sum(a * b for a, b in zip(sizes[:-1], sizes[1:])) + sizes[-1]
    bwd = sum(a * b for a, b in zip(sizes[:-1], sizes[1:]))
    return 2 * (fwd + bwd)


def flops_model(n_rad, n_eta, pairs, triplets, triplets_in):
    """Algorithmic FLOPs of the descriptor forward and adjoint passes.

    Counted from the definitions, one FLOP per add, multiply, square root,
    exponential or cosine:
      forward  per pair:    displacement 3, r 6, f_c 4, exp(-eta r^2) f_c 3 n_eta, radial 6 n_rad
               per triplet: r_jk^2 and the cutoff test 9;  in range: r_jk 1, f_c 4, cos 7,
                            (1 +- cos)^zeta 8, per eta: exp 2, product 3, 8 features x 2
      adjoint  per pair:    forward pair terms + derivative factors 2 n_eta + radial derivative
                            10 n_rad + slot vector 4 + virial 18
               per triplet: test 9;  in range: r_jk and 1/r_jk 2, f_c and f_c' 7, cos 7,
                            powers and their derivatives 14, per eta: exp 2, S 16, S' 16,
                            four partials 14, gradient coefficients 10, two vectors 24,
                            slot accumulation 6
    """
    fwd_pair = 13 + 3 * n_eta + 6 * n_rad
    fwd_trip_in = 20 + 21 * n_eta
    adj_pair = fwd_pair + 2 * n_eta + 10 * n_rad + 22
    adj_trip_in = 30 + 48 * n_eta + 40
    fwd = pairs * fwd_pair + triplets * 9 + triplets_in * fwd_trip_in
    adj = pairs * adj_pair + triplets * 9 + triplets_in * adj_trip_in
    return fwd, adj


def g5_flops_model(n_rad, n_eta, n_el, slots, centres):
    """Algorithmic FLOPs of the G5 forward and adjoint passes (spherical-harmonic
    moments up to l = 8: 81 harmonics, 45 (l, m >= 0) recursion steps), counted
    like flops_model (a fused multiply-add is two):
      forward  per slot:   the G4 pair terms (13 + 3 n_eta + 6 n_rad); (x + iy)^m 48;
                           recursion 45 x 4; harmonics 81; per eta and harmonic:
                           M += w Y 2, R += (w Y)^2 3
               per centre: per element pair and eta: power spectrum 81 x 3,
                           8 features x 18
      adjoint  per slot:   the G4 adjoint pair terms (fwd pair + 2 n_eta + 10 n_rad + 22);
                           (x + iy)^m 48; recursion with z derivative 45 x 8; per eta:
                           six (four for m = 0) accumulations per (l, m) 9 x 8 + 36 x 12,
                           fold per m 9 x 20; tangent projection and vector 30; virial 18
               per centre: H 9 x 16 and dE/dM 81 x 2 n_el per element pair / element and eta
    """
    n_pairs = n_el * (n_el + 1) // 2
    fwd_slot = 13 + 3 * n_eta + 6 * n_rad + 48 + 180 + 81 + 81 * 5 * n_eta
    fwd_centre = n_pairs * n_eta * (81 * 3 + 8 * 18)
    adj_slot = (13 + 3 * n_eta + 6 * n_rad) + 2 * n_eta + 10 * n_rad + 22 + 48 + 360 + \
        n_eta * (9 * 8 + 36 * 12 + 9 * 20) + 30 + 18
    adj_centre = n_pairs * n_eta * 9 * 16 + n_el * n_eta * 81 * 2 * n_el
    return slots * fwd_slot + centres * fwd_centre, slots * adj_slot + centres * adj_centre


def gfn_flops_per_edge(n_rad, H, L):
    """Algorithmic FLOPs of the direct-force head per directed edge, counted
    from its definition (one FLOP per add, multiply, exp or divide; tanh 5):
    radial basis 6 n_rad and e^(0) 2 H n_rad; an H->H->H MLP 4 H^2 + 7 H;
    layer l rebuilds e^(l) (l edge MLPs on n_i + n_j, H adds each) and applies
    the message MLP (+H to accumulate); the readout rebuilds e^(L) and applies
    phi_f (2 H^2 + 7 H) and the edge force (6).  Returns (layers, readout)."""
    basis = 6 * n_rad + 2 * H * n_rad
    mlp = 4 * H * H + 7 * H
    layers = sum(basis + l * (mlp + 2 * H) + mlp + H for l in range(L))
    readout = basis + L * (mlp + 2 * H) + 2 * H * H + 7 * H + 6
    return layers, readout


def xrd_flops_per_pair(periodic):
    """Algorithmic FLOP of one ordered pair of the XRD CV sum and its gradient,
    one per add, multiply, rounding, sqrt, division, sin or cos: displacement 3,
    minimum image 3 x 3, r^2 5, r 1, x = Q r 1, sin and cos 2, sinc = sin/x 1,
    f_j sinc accumulated 2, (cos - sinc)/r^2 2, times f_j 1, gradient
    accumulated 3 x 2."""
    return 3 + (9 if periodic else 0) + 5 + 1 + 1 + 2 + 1 + 2 + 2 + 1 + 6


def metad_report(eng, wl, spec, n_reps):
    """Bias-pass timing and, for the XRD CV, the roofline of its all-pairs kernel."""
    bias_ms = eng.time_bias(n_reps)
    out = {"cv": spec.cv, "stride": spec.stride, "sigma": spec.sigma, "bias_factor": spec.gamma,
           "height0_eV": spec.height0, "bias_pass_ms": round(bias_ms, 4)}
    if spec.cv == "xrd":
        pairs = sum(s.n_beads * s.n_atoms * s.n_atoms for s in wl.systems)
        periodic = any(float(b) > 0 for s in wl.systems for b in s.box)
        flops = pairs * xrd_flops_per_pair(periodic)
        achieved = flops / (bias_ms * 1e-3) / 1e12
        out["roofline"] = {"kernel": "k_xrd_rows + k_metad_bias (all-pairs XRD CV, FP64)", "bound": "alu",
                           "achieved": round(achieved, 3), "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                           "flops_per_launch": flops, "launch_ms": round(bias_ms, 4),
                           "work": {"ordered_pairs": pairs, "flops_per_pair": xrd_flops_per_pair(periodic)}}
    return out


def time_steps(eng, steps, warmup, restart=None):
    """Wall and GPU-event seconds of `steps` steps after `warmup`.  With
    restart = (q0, p0, every) the steps run in blocks of `every`, each from
    the initial state (set between blocks, outside the timed spans), and the
    block times are summed: a head without an energy is not conservative, and
    with random weights it heats the ring without bound over hundreds of steps."""
    import torch
    eng.step(warmup)
    torch.cuda.synchronize()
    blocks = [steps] if restart is None else [min(restart[2], steps - k) for k in range(0, steps, restart[2])]
    wall = gpu = 0.0
    for n in blocks:
        if restart is not None:
            eng.set_state(restart[0], restart[1])
            torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record(eng.stream)
        eng.step(n)
        stop.record(eng.stream)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        gpu += start.elapsed_time(stop) / 1e3
    eng.estimators()            # raises if a neighbour list overflowed in the timed steps
    return wall, gpu


def plain_fp32(wl, steps, warmup, device, shape=None, skin=0.0):
    """The comparison path: FP32 MLP, no graph, one context per system (with the
    launch shape and neighbour lists of the timed path, so the two differ only
    in MLP precision, batching and graph replay)."""
    import torch
    from paper_2503_23728_amd import synthetic as S
    from paper_2503_23728_amd.pimd import Pimd
    q, p = S.initial_state(wl)
    engines = []
    off = 0
    for s in wl.systems:
        n = s.n_atoms * s.n_beads
        e = Pimd([s], wl.model, wl.dt, wl.tau0, wl.pile_lambda, wl.philox_seed, precision="fp32", device=device,
                 potential="gfn" if hasattr(wl.model, "width") else "bpnn",
                 neighbor_skin=skin if np.any(np.asarray(s.box) > 0) else 0.0)
        e.set_graph(False)
        if shape is not None:   # the same shape; the register-chained MLP is a BF16 kernel
            e.set_tuning(**dict(shape, mlp_chain=0))
        e.set_state(torch.from_numpy(q[off:off + n]).to(device), torch.from_numpy(p[off:off + n]).to(device))
        engines.append(e)
        off += n
    for e in engines:
        e.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for e in engines:
            e.step(1)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def force_error(F, F_ref):
    """max_i |F_i - F_i^ref| / max(|F_i^ref|, 0.1 F_rms^ref): the parity tests' metric."""
    F = np.asarray(F, dtype=np.float64).reshape(-1, 3)
    F_ref = np.asarray(F_ref, dtype=np.float64).reshape(-1, 3)
    nref = np.linalg.norm(F_ref, axis=1)
    floor = 0.1 * np.sqrt(np.mean(nref ** 2))
    return float(np.max(np.linalg.norm(F - F_ref, axis=1) / np.maximum(nref, floor)))


def cpu_baseline(wl, budget_s=20.0, gpu_forces=None):
    """FP64 oracle on the host cores over a bounded sample of the workload:
    whole integrator steps of the first ring polymer(s), repeated until about
    budget_s seconds have passed; when one step of the first ring polymer is
    itself too large for that (more than 20,000 bead-atoms), force evaluations
    of its beads one at a time (every atom of a bead with all its neighbours;
    the integrator is a few percent of a step on either side).  gpu_forces:
    the benchmarked path's forces at the same initial state, compared with the
    oracle's forces of the sample (force_err_vs_fp64)."""
    from paper_2503_23728_amd import synthetic as S
    from oracle import bpnn, gfn, ring
    q, p = S.initial_state(wl)
    first = wl.systems[0]
    cores = len(os.sched_getaffinity(0))
    threads = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    if first.n_atoms * first.n_beads > 20000:
        n_at = first.n_atoms
        t0 = time.perf_counter()
        k = 0
        err = 0.0
        while True:
            qb = q[k * n_at:(k + 1) * n_at]
            if hasattr(wl.model, "width"):
                sub = S.Workload(wl.name, [S.System(n_at, 1, first.temperature, first.box, first.species,
                                                    first.q0)], wl.model, wl.dt, wl.tau0, wl.pile_lambda,
                                 wl.n_steps, wl.philox_seed, wl.momentum_seed)
                F_ref = gfn.forces(sub, qb)
            else:
                F_ref = bpnn.bead_energy_forces(wl.model, qb, first.species, first.box)[1]
            if gpu_forces is not None:
                err = max(err, force_error(gpu_forces[k * n_at:(k + 1) * n_at], F_ref))
            k += 1
            if time.perf_counter() - t0 > budget_s or k >= first.n_beads:
                break
        dt = time.perf_counter() - t0
        out = dict(value=n_at * k / dt, unit="bead-atom force evals/s", cores=threads, kind="oracle",
                   sample=f"{k} FP64 oracle force evaluations of whole beads of {n_at} atoms "
                          f"({n_at * k} bead-atoms, {dt:.1f} s)")
        if gpu_forces is not None:
            out["force_err_vs_fp64"] = {"value": err, "sample": f"every atom of beads 0-{k - 1} at the initial state"}
        return out
    systems, rows, n_sys = [], 0, 0
    for s in wl.systems:
        systems.append(s)
        rows += s.n_atoms * s.n_beads
        n_sys += 1
        if rows >= 1000 or n_sys >= 16:
            break
    sub = S.Workload(wl.name, systems, wl.model, wl.dt, wl.tau0, wl.pile_lambda, wl.n_steps, wl.philox_seed,
                     wl.momentum_seed)

    def fn(qq):
        if hasattr(wl.model, "width"):
            return np.zeros(sum(s.n_beads for s in systems)), gfn.forces(sub, qq.astype(np.float32))
        E, F, _ = bpnn.energy_forces(sub, qq.astype(np.float32))
        return E, F
    rp = ring.RingPolymers([(s.n_atoms, s.n_beads, s.temperature, wl.model.masses[s.species]) for s in systems],
                           wl.dt, wl.tau0, wl.pile_lambda, wl.philox_seed, fn)
    rp.set_state(q[:rows].astype(np.float64), p[:rows].astype(np.float64))
    err = force_error(gpu_forces[:rows], fn(q[:rows])[1]) if gpu_forces is not None else None
    t0 = time.perf_counter()
    n = 0
    while True:
        rp.step()
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 200:
            break
    dt = time.perf_counter() - t0
    out = dict(value=rows * n / dt, unit="bead-atom force evals/s", cores=threads, kind="oracle",
               sample=f"{n} FP64 oracle integrator steps of {len(systems)} ring polymer(s), {rows} bead-atoms "
                      f"({dt:.1f} s)")
    if err is not None:
        out["force_err_vs_fp64"] = {"value": err, "sample": f"every bead-atom of the first {len(systems)} ring "
                                                            f"polymer(s) at the initial state"}
    return out


def extra_keys(args, wl, eng, skin, shape, device):
    """The same workload with per-bead cell searches every step (no shared
    lists), the same workload on float32-valued weights, and the batched workload 4 (512 ring polymers in one graph per step)
    against its plain-FP32 path (one eager context per ring polymer)."""
    import torch
    from paper_2503_23728_amd import synthetic as S
    from paper_2503_23728_amd.pimd import Pimd
    out = {}
    q, p = S.initial_state(wl)
    if skin > 0:
        cell = Pimd.from_workload(wl, precision=args.precision, device=device, transform=args.transform)
        cell.set_state(torch.from_numpy(q).to(device), torch.from_numpy(p).to(device))
        if not args.no_tune:
            cell.autotune(n_reps=3)
        wall, _ = time_steps(cell, args.steps, args.warmup)
        out["cell_search_every_step"] = {"value": wl.bead_atoms * args.steps / wall,
                                         "ms_per_step": 1e3 * wall / args.steps,
                                         "neighbor_lists": "per bead, cell search every evaluation"}
        print(f"[bench] cell search every step: {1e3 * wall / args.steps:.3f} ms/step", file=sys.stderr,
              flush=True)
        cell.close()
        del cell
    if args.precision == "bf16":
        # the same systems on weights with float32 mantissas (a model trained in
        # FP32): the split BF16 MLP then splits the weights too, three products
        # per term instead of two; same launch shape
        fwl = S.workload(args.config, bf16_weights=False)
        f32w = Pimd.from_workload(fwl, precision="bf16", device=device, transform=args.transform,
                                  neighbor_skin=skin)
        f32w.set_state(torch.from_numpy(q).to(device), torch.from_numpy(p).to(device))
        f32w.set_tuning(**shape)
        wall, _ = time_steps(f32w, args.steps, args.warmup)
        kern = f32w.time_stages(max(args.profile_reps, 5))
        out["float32_valued_weights"] = {"value": wl.bead_atoms * args.steps / wall,
                                         "ms_per_step": 1e3 * wall / args.steps,
                                         "mlp_ms": round(kern["mlp"], 4),
                                         "mlp": "activations and weights split, three BF16 products per term"}
        print(f"[bench] float32-valued weights: {1e3 * wall / args.steps:.3f} ms/step, MLP "
              f"{kern['mlp']:.4f} ms", file=sys.stderr, flush=True)
        f32w.close()
        del f32w
    if args.config != 4:
        bwl = S.workload(4)
        bat = Pimd.from_workload(bwl, precision=args.precision, device=device)
        bq, bp = S.initial_state(bwl)
        bat.set_state(torch.from_numpy(bq).to(device), torch.from_numpy(bp).to(device))
        bshape = bat.get_tuning() if args.no_tune else bat.autotune(n_reps=3)[0]
        wall, _ = time_steps(bat, args.steps, args.warmup)
        bat.close()
        del bat
        psteps = max(1, min(args.steps, 50))
        pwall = plain_fp32(bwl, psteps, min(args.warmup, 5), device, bshape, 0.0)
        val, pval = bwl.bead_atoms * args.steps / wall, bwl.bead_atoms * psteps / pwall
        out["batched_workload"] = {"workload": bwl.name, "bead_atoms": bwl.bead_atoms, "value": val,
                                   "ms_per_step": 1e3 * wall / args.steps,
                                   "plain_fp32": {"value": pval, "steps": psteps,
                                                  "ms_per_step": 1e3 * pwall / psteps,
                                                  "launch": "eager, one context per system"},
                                   "vs_plain_fp32": val / pval}
        print(f"[bench] batched {bwl.name}: {1e3 * wall / args.steps:.3f} ms/step, plain fp32 "
              f"{1e3 * pwall / psteps:.3f} ms/step", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "bf16-plain"])
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-FP32 comparison path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra keys (per-step cell search; batched workload 4 against plain FP32)")
    ap.add_argument("--profile-reps", type=int, default=10)
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shape (no autotuner)")
    ap.add_argument("--potential", default="bpnn", choices=["bpnn", "gfn"],
                    help="energy model with adjoint forces, or the direct-force head")
    ap.add_argument("--gfn-width", type=int, default=16)
    ap.add_argument("--gfn-layers", type=int, default=2)
    ap.add_argument("--transform", default="normal-modes", choices=["normal-modes", "staging", "primitive"],
                    help="ring-polymer coordinates of the integrator")
    ap.add_argument("--angular", default="g4", choices=["g4", "g5"],
                    help="angular symmetry functions: G4 (triplets within the cutoff) or G5 (no r_jk "
                         "factors, summed through spherical-harmonic moments)")
    ap.add_argument("--skin", type=float, default=None,
                    help="neighbour lists shared by the beads of a ring polymer: centroid lists with this skin "
                         "(A), filtered per bead (the same lists); 0 searches every bead's cells each step; "
                         "ignored for systems without a box.  Default 2 for the energy model, 0 for the "
                         "direct-force head (its random weights heat the rings past any skin)")
    ap.add_argument("--metad", action="store_true",
                    help="add the well-tempered metadynamics bias of the workload's study (s_dimer or XRD CV)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described in the design notes, not built)"}))
        sys.exit(2)

    import torch
    from paper_2503_23728_amd import synthetic as S
    from paper_2503_23728_amd.pimd import Pimd

    device = "cuda:0"
    gfn_mode = args.potential == "gfn"
    wl = S.gfn_workload(args.config, args.gfn_width, args.gfn_layers) if gfn_mode else S.workload(args.config)
    if args.angular == "g5":
        if gfn_mode:
            sys.exit("--angular g5 applies to the energy model only")
        wl = S.with_g5(wl)
    B = wl.bead_atoms
    spec = S.metad_spec(wl, max_hills=4096) if args.metad else None
    skin = args.skin if args.skin is not None else (0.0 if gfn_mode else 2.0)
    skin = skin if all(np.any(np.asarray(s.box) > 0) for s in wl.systems) else 0.0
    eng = Pimd.from_workload(wl, precision=args.precision, device=device, metad=spec, transform=args.transform,
                             neighbor_skin=skin)
    q, p = S.initial_state(wl)
    eng.set_state(torch.from_numpy(q).to(device), torch.from_numpy(p).to(device))
    if args.no_tune:
        shape, cached = eng.get_tuning(), None
    else:
        t0 = time.perf_counter()
        shape, cached = eng.autotune(n_reps=3)
        print(f"[bench] launch shape {shape} ({'cached' if cached else 'autotuned'} in "
              f"{time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    print(f"[bench] {wl.name}: {B} bead-atoms, {len(wl.systems)} systems; warmup {args.warmup}", file=sys.stderr,
          flush=True)
    restart = None
    if gfn_mode:
        restart = (torch.from_numpy(q).to(device), torch.from_numpy(p).to(device), 25)
    wall, gpu_s = time_steps(eng, args.steps, args.warmup, restart)
    ms_per_step = 1e3 * wall / args.steps
    value = B * args.steps / wall
    ns_day = args.steps * wl.dt * 1e-6 / wall * 86400.0
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    # per-stage timing with HIP events on the launch stream (kernels one by one,
    # one integrator step per repetition) and gap-free kernel timing (each force
    # stage enqueued back to back on the current positions)
    stages = eng.profile_stages(args.profile_reps)
    kern = eng.time_stages(max(args.profile_reps, 5))
    pairs, trip, trip_in = eng.work_counts()
    m = wl.model
    if gfn_mode:
        kern = {"neighbors": kern["neighbors"], "gfn_layers": kern["descriptors"], "gfn_readout": kern["adjoint"],
                "bead_sums": kern["forces"]}
        lf, rf = gfn_flops_per_edge(m.n_rad, m.width, m.n_layers)
        flops = pairs * (lf + rf) + B * m.n_layers * (6 * m.width * m.width + 7 * m.width)
        head_ms = kern["gfn_layers"] + kern["gfn_readout"]
        achieved = flops / (head_ms * 1e-3) / 1e12
        roofline = {"kernel": "k_gfn_layer + k_gfn_forces (direct-force head)", "bound": "alu",
                    "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                    "flops_per_launch": flops, "launch_ms": round(head_ms, 4),
                    "work": {"pairs": pairs, "width": m.width, "layers": m.n_layers}}
    elif args.angular == "g5":
        # the forward (FP64 moment sums) is the dominant kernel; FP64 and unpacked
        # FP32 vector instructions issue at the same rate, 78.6 TFLOP/s
        fwd_flops, adj_flops = g5_flops_model(m.n_rad, len(m.ang_eta), m.n_elements, pairs, B)
        fwd_ms, adj_ms = kern["descriptors"], kern["adjoint"]
        achieved = fwd_flops / (fwd_ms * 1e-3) / 1e12
        mlp_flops = B * mlp_flops_per_row(eng.D, m.hidden)
        roofline = {"kernel": "k_descriptors_g5 (spherical-harmonic moments, FP64 sums)", "bound": "alu",
                    "achieved": round(achieved, 3), "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                    "flops_per_launch": fwd_flops, "launch_ms": round(fwd_ms, 4),
                    "adjoint": {"kernel": "k_adjoint_g5", "flops_per_launch": adj_flops,
                                "launch_ms": round(adj_ms, 4),
                                "achieved": round(adj_flops / (adj_ms * 1e-3) / 1e12, 3)},
                    "mlp": {"kernel": "k_mlp", "bound": "mfma", "flops_per_launch": mlp_flops,
                            "launch_ms": round(kern["mlp"], 4),
                            "achieved": round(mlp_flops / (kern["mlp"] * 1e-3) / 1e12, 3),
                            "peak": BF16_MFMA_PEAK_TFLOPS,
                            "frac": round(mlp_flops / (kern["mlp"] * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4)},
                    "work": {"slots": pairs, "centres": B}}
    else:
        fwd_flops, adj_flops = flops_model(m.n_rad, len(m.ang_eta), pairs, trip, trip_in)
        adj_ms = kern["adjoint"]
        achieved = adj_flops / (adj_ms * 1e-3) / 1e12
        traffic = measured_traffic(wl.name)
        mlp_flops = B * mlp_flops_per_row(eng.D, m.hidden)
        roofline = {"kernel": "k_adjoint (descriptor adjoint with recomputation)", "bound": "alu",
                    "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": traffic,
                    "flops_per_launch": adj_flops, "launch_ms": round(adj_ms, 4),
                    "forward": {"kernel": "k_descriptors", "flops_per_launch": fwd_flops,
                                "launch_ms": round(kern["descriptors"], 4),
                                "achieved": round(fwd_flops / (kern["descriptors"] * 1e-3) / 1e12, 3)},
                    "mlp": {"kernel": "k_mlp", "bound": "mfma", "flops_per_launch": mlp_flops,
                            "launch_ms": round(kern["mlp"], 4),
                            "achieved": round(mlp_flops / (kern["mlp"] * 1e-3) / 1e12, 3),
                            "peak": BF16_MFMA_PEAK_TFLOPS,
                            "frac": round(mlp_flops / (kern["mlp"] * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4)},
                    "work": {"pairs": pairs, "triplets": trip, "triplets_in_range": trip_in}}
    print(f"[bench] stages {json.dumps({k: round(v, 4) for k, v in stages.items()})}", file=sys.stderr, flush=True)
    print(f"[bench] kernels {json.dumps({k: round(v, 4) for k, v in kern.items()})}", file=sys.stderr, flush=True)

    out = {
        "metric": "bead·atom force evals/s + PIMD ns/day vs plain FP32, at force err vs FP64",
        "value": value, "unit": "bead-atom force evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "f32 (MLP GEMM operands bf16: activations split in hi + lo parts, "
                                         "weights bfloat16 values)",
                  "bf16-plain": "f32 (MLP GEMM operands bf16)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": wl.name, "systems": len(wl.systems), "bead_atoms": B,
                   "beads": sum(s.n_beads for s in wl.systems), "dt_fs": wl.dt,
                   "precision": args.precision, "potential": args.potential, "angular": args.angular,
                   "transform": args.transform,
                   "launch": "hip graph per step" + (", 25-step blocks from the initial state" if gfn_mode else ""),
                   "launch_shape": shape,
                   "neighbor_lists": (f"shared by the beads: centroid lists, skin {skin} A, "
                                      f"{eng.neighbor_rebuilds()[0]} builds in {args.warmup + args.steps} steps + "
                                      f"profiling" if skin > 0 else "per bead, cell search every evaluation"),
                   "shape_source": {None: "default", True: "tuning cache", False: "autotuner"}[cached]},
        "ns_per_day": ns_day, "gpu_event_s": gpu_s,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "kernel_ms": {k: round(v, 4) for k, v in kern.items()},
        "roofline": roofline,
    }
    if not args.no_plain:
        psteps = max(1, min(args.steps, 50 if len(wl.systems) > 1 else args.steps))
        pwall = plain_fp32(wl, psteps, min(args.warmup, 5), device, shape, skin)
        pval = B * psteps / pwall
        out["plain_fp32"] = {"value": pval, "steps": psteps, "ms_per_step": 1e3 * pwall / psteps,
                             "launch": "eager, one context per system"}
        out["vs_plain_fp32"] = value / pval
        print(f"[bench] plain fp32: {1e3 * pwall / psteps:.3f} ms/step", file=sys.stderr, flush=True)
    if gfn_mode:
        # the energy model with adjoint forces on the same systems (BF16-split MLP, its own tuned
        # shape, the shared skin lists of the default run where the systems are periodic)
        ewl = S.workload(args.config)
        eskin = 2.0 if all(np.any(np.asarray(s.box) > 0) for s in ewl.systems) else 0.0
        eeng = Pimd.from_workload(ewl, precision="bf16", device=device, neighbor_skin=eskin)
        eq, ep = S.initial_state(ewl)
        eeng.set_state(torch.from_numpy(eq).to(device), torch.from_numpy(ep).to(device))
        if not args.no_tune:
            eeng.autotune(n_reps=3)
        ewall, _ = time_steps(eeng, args.steps, args.warmup)
        out["energy_model_ms_per_step"] = 1e3 * ewall / args.steps
        out["energy_model_neighbor_lists"] = (f"shared by the beads: centroid lists, skin {eskin} A" if eskin > 0
                                              else "per bead, cell search every evaluation")
        out["head_speedup_vs_energy_model"] = ewall / wall
        print(f"[bench] energy model: {1e3 * ewall / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    if spec is not None:
        out["metad"] = metad_report(eng, wl, spec, max(args.profile_reps, 5))
        out["config"]["workload"] += f"+wt-metad({spec.cv})"
        print(f"[bench] metad {json.dumps(out['metad'])}", file=sys.stderr, flush=True)
    if not args.no_extras and not gfn_mode and not args.metad and args.angular == "g4":
        out.update(extra_keys(args, wl, eng, skin, shape, device))
    if not args.no_cpu:
        # the benchmarked path's forces at the initial state, for the oracle sample to check
        # (the potential alone: not with a metadynamics bias)
        F_init = None
        if spec is None:
            q_init, _ = S.initial_state(wl)
            F_init = eng.energy_forces(torch.from_numpy(q_init).to(device))[1].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(wl, gpu_forces=F_init)
        if "force_err_vs_fp64" in out["cpu_baseline"]:
            out["force_err_vs_fp64"] = dict(out["cpu_baseline"]["force_err_vs_fp64"],
                                            metric="max_i |F_i - F_i^FP64| / max(|F_i^FP64|, 0.1 F_rms)")
            print(f"[bench] force err vs FP64 {out['force_err_vs_fp64']['value']:.2e}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
