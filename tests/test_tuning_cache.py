"""Host logic of the launch-shape cache (no GPU)."""
import json

from paper_2503_23728_amd import synthetic as S
from paper_2503_23728_amd import tuning


def _key(wl, **kw):
    args = dict(arch="gfx950", n_cu=256, systems=wl.systems, model=wl.model, precision="bf16", max_neighbors=0)
    args.update(kw)
    return tuning.config_key(**args)


def test_key_is_stable_and_sensitive_to_what_the_shape_depends_on():
    wl = S.small_workload("water8", n_beads=4)
    k = _key(wl)
    assert k == _key(S.small_workload("water8", n_beads=4))
    assert k != _key(wl, precision="fp32")
    assert k != _key(wl, arch="gfx942")
    assert k != _key(wl, n_cu=304)
    assert k != _key(S.small_workload("water8", n_beads=8))
    assert k != _key(wl, max_neighbors=64)


def test_key_separates_the_angular_form_and_the_shared_lists():
    wl = S.workload(2)
    base = _key(wl)
    assert _key(S.with_g5(wl)) != base
    assert _key(wl, neighbor_skin=2.0) != base
    assert _key(wl, neighbor_skin=2.0) != _key(wl, neighbor_skin=3.0)
    assert _key(wl, neighbor_skin=0.0) == base


def test_key_ignores_system_order():
    wl = S.workload(4)
    a = tuning.config_key("gfx950", 256, wl.systems, wl.model, "bf16", 0)
    b = tuning.config_key("gfx950", 256, list(reversed(wl.systems)), wl.model, "bf16", 0)
    assert a == b


def test_store_and_load_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "t.json")
    assert tuning.load("k", path) is None
    shape = {"centre_waves": 2, "centre_grid": 0, "mlp_rows": 32, "neighbor_cells": 1, "mlp_waves": 8,
             "force_rows": 1, "centre_lanes": 0, "mlp_chain": 0}
    assert tuning.store("k", shape, path)
    assert tuning.load("k", path) == shape
    assert tuning.store("k2", {"centre_waves": 4, "centre_grid": 512, "mlp_rows": 16, "neighbor_cells": 0,
                               "mlp_waves": 4, "force_rows": 0, "centre_lanes": 1, "mlp_chain": 1}, path)
    assert tuning.load("k", path)["mlp_rows"] == 32
    assert set(json.load(open(path))) == {"k", "k2"}


def test_corrupt_or_partial_entries_are_ignored(tmp_path):
    path = tmp_path / "t.json"
    path.write_text("not json")
    assert tuning.load("k", str(path)) is None
    path.write_text(json.dumps({"k": {"centre_waves": 2}}))
    assert tuning.load("k", str(path)) is None
    # an entry written before a field existed is not applied
    path.write_text(json.dumps({"k": {"centre_waves": 2, "centre_grid": 0, "mlp_rows": 16, "neighbor_cells": 0}}))
    assert tuning.load("k", str(path)) is None
    assert tuning.store("k", {"centre_waves": 1, "centre_grid": 0, "mlp_rows": 64, "neighbor_cells": 0,
                              "mlp_waves": 4, "force_rows": 1, "centre_lanes": 0, "mlp_chain": 0}, str(path))
    assert tuning.load("k", str(path))["centre_waves"] == 1


def test_key_of_the_direct_force_head_differs_from_the_energy_model():
    wl = S.workload(2)
    head = S.gfn_workload(2)
    a = tuning.config_key("gfx950", 256, wl.systems, wl.model, "fp32", 0)
    b = tuning.config_key("gfx950", 256, head.systems, head.model, "fp32", 0)
    c = tuning.config_key("gfx950", 256, head.systems, S.gfn_workload(2, width=32).model, "fp32", 0)
    assert len({a, b, c}) == 3
