"""pimd_init_static, the allocation-free pimd_init: contexts on the library's
own static device workspace give bitwise the results of contexts on a caller
workspace (forces, energies, virials, integrator steps with injected and
Philox noise, estimators).  Two static contexts run in a row on one device,
the second on a smaller system, so it starts from the array the first left
behind.  Sizes beyond the array and a second live static context are refused.
"""
import sys

import numpy as np
import pytest

from paper_2503_23728_amd import abi
from paper_2503_23728_amd import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(wl, static, skin):
    from paper_2503_23728_amd.pimd import Pimd
    eng = Pimd.from_workload(wl, device="cuda:0", precision="bf16", static_workspace=static, regrow=False,
                             neighbor_skin=skin)
    q = torch.from_numpy(S.perturbed_beads(wl, 0.05, seed=11)).cuda()
    _, p0 = S.initial_state(wl)
    p = torch.from_numpy(p0).cuda()
    xi = torch.from_numpy(np.random.default_rng(12).normal(size=(2, len(p0), 3)).astype(np.float32)).cuda()
    E, F, W = eng.energy_forces(q, virial=True)
    out = [E.cpu().numpy(), F.cpu().numpy(), W.cpu().numpy()]
    eng.set_state(q, p)
    eng.inject_noise(xi)
    eng.step(1)
    eng.step(6)
    qs, ps, Fs, step = eng.get_state()
    est = eng.estimators()[0]
    out += [qs.cpu().numpy(), ps.cpu().numpy(), Fs.cpu().numpy(), np.array([step]),
            np.array([est[k] for k in ("V_bar", "K_prim", "K_cv", "E_spring", "K_beads", "H_conserved")])]
    eng.close()
    return out


@pytest.mark.parametrize("kind,beads,skin", [("water8", 8, 2.0), ("fad", 4, 0.0)])
def test_static_workspace_gives_the_caller_workspace_results(kind, beads, skin):
    # water 8 (8 beads, shared lists) first, then the smaller formic acid dimer
    wl = S.small_workload(kind, n_beads=beads)
    say(f"static workspace: {kind} P={beads} skin={skin}")
    got = _run(wl, True, skin)
    want = _run(wl, False, skin)
    for name, a, b in zip(("E", "F", "W", "q", "p", "F_state", "step", "estimators"), got, want):
        assert np.all(np.isfinite(a)), name
        assert np.array_equal(a, b), (name, np.max(np.abs(a - b)))


def test_static_workspace_refuses_what_it_cannot_hold():
    from paper_2503_23728_amd.pimd import Pimd, make_config
    wl = S.workload(2)            # water 64, P = 32: about 130 MiB of workspace
    cfg, keep = make_config(wl.systems, wl.model, wl.dt, wl.tau0, wl.pile_lambda, wl.philox_seed, "bf16", "bpnn",
                            0.0, 0, None, None, "normal-modes", 0.0)
    st, need = abi.pimd_workspace_size(cfg)
    assert st == abi.PIMD_OK and need > abi.PIMD_STATIC_WORKSPACE_BYTES
    st, ctx = abi.pimd_init_static(cfg, torch.cuda.current_stream().cuda_stream)
    assert st == abi.PIMD_E_CAPACITY and not ctx
    assert "static workspace" in abi.pimd_last_error(None)
    # one static context per device at a time; closing it frees the array
    small = S.small_workload("fad", n_beads=4)
    a = Pimd.from_workload(small, device="cuda:0", static_workspace=True)
    cfg2, keep2 = make_config(small.systems, small.model, small.dt, small.tau0, small.pile_lambda,
                              small.philox_seed, "fp32", "bpnn", 0.0, 0, None, None, "normal-modes", 0.0)
    st, ctx = abi.pimd_init_static(cfg2, torch.cuda.current_stream().cuda_stream)
    assert st == abi.PIMD_E_STATE and not ctx
    a.close()
    b = Pimd.from_workload(small, device="cuda:0", static_workspace=True)
    E, F, _ = b.energy_forces(torch.from_numpy(S.perturbed_beads(small, 0.05, seed=3)).cuda())
    assert np.all(np.isfinite(F.cpu().numpy()))
    b.close()
