"""GPU: checkpoint and restore are bitwise.

The thermostat noise is a counter-based stream (Philox keyed by the seed,
counted by step, row and half-step), the forces of a state are a
deterministic function of its positions, and the neighbour lists are exact
whichever way they are built, so a context that is given a saved
(positions, momenta, step) continues exactly as the one that saved it.
"""
import sys

import pytest

from paper_2503_23728_amd import synthetic as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _engine(wl, **kw):
    from paper_2503_23728_amd.pimd import Pimd
    return Pimd.from_workload(wl, device="cuda:0", **kw)


CASES = {
    "water64-nm-skin": (lambda: S.workload(2), dict(precision="bf16", neighbor_skin=2.0)),
    "water64-staging": (lambda: S.workload(2), dict(precision="bf16", transform="staging")),
    "fad-primitive": (lambda: S.small_workload("fad", n_beads=8), dict(precision="fp32", transform="primitive")),
    "water64-g5": (lambda: S.with_g5(S.workload(2)), dict(precision="bf16", neighbor_skin=2.0)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_restored_context_continues_bitwise(name):
    make, kw = CASES[name]
    wl = make()
    say(f"checkpoint {name}")
    q0, p0 = S.initial_state(wl)
    a = _engine(wl, **kw)
    a.set_state(torch.from_numpy(q0).cuda(), torch.from_numpy(p0).cuda(), step=0)
    a.step(25)
    q, p, _, step = a.get_state()
    saved = (q.clone(), p.clone(), step)
    a.step(25)
    qa, pa, Fa, sa = a.get_state()
    b = _engine(wl, **kw)
    b.set_state(saved[0], saved[1], step=saved[2])
    b.step(25)
    qb, pb, Fb, sb = b.get_state()
    assert saved[2] == 25 and sa == sb == 50
    assert torch.equal(qa, qb) and torch.equal(pa, pb) and torch.equal(Fa, Fb)
