"""The C-ABI library loads without a GPU, exports every function the header
declares, and rejects bad arguments with the documented status before any
HIP call."""
import ctypes

import numpy as np
import pytest

from paper_2503_23728_amd import abi, synthetic as S
from paper_2503_23728_amd.pimd import make_config


@pytest.fixture(scope="module")
def lib():
    return abi.lib()


def test_exports_every_declared_function(lib):
    names = abi.declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(abi._SIGNATURES)


def test_status_strings(lib):
    for s in range(8):
        assert abi.pimd_status_str(s)
    assert abi.pimd_status_str(99) == "unknown status"


def _cfg(wl, **kw):
    return make_config(wl.systems, wl.model, wl.dt, wl.tau0, wl.pile_lambda, wl.philox_seed, **kw)


def test_workspace_size_of_valid_configs(lib):
    for c in (1, 2, 3):
        cfg, keep = _cfg(S.workload(c))
        st, n = abi.pimd_workspace_size(cfg)
        assert st == abi.PIMD_OK and n > 0


def test_workspace_grows_with_max_neighbors(lib):
    wl = S.workload(2)
    a = abi.pimd_workspace_size(_cfg(wl, max_neighbors=64)[0])[1]
    b = abi.pimd_workspace_size(_cfg(wl, max_neighbors=256)[0])[1]
    assert b > a


def test_skin_configs(lib):
    # shared centroid lists: a box for every system, skin >= 0; their buffers sized per atom
    wl = S.workload(2)
    a = abi.pimd_workspace_size(_cfg(wl)[0])[1]
    st, b = abi.pimd_workspace_size(_cfg(wl, neighbor_skin=2.0)[0])
    n = wl.systems[0].n_atoms
    assert st == abi.PIMD_OK and n * (3 * 128 * 4 + 40) <= b - a <= n * (3 * 128 * 4 + 40) + 4096
    assert abi.pimd_workspace_size(_cfg(wl, neighbor_skin=-1.0)[0])[0] == abi.PIMD_E_ARG
    assert abi.pimd_workspace_size(_cfg(wl, neighbor_skin=float("nan"))[0])[0] == abi.PIMD_E_ARG
    fad = S.workload(1)
    assert abi.pimd_workspace_size(_cfg(fad, neighbor_skin=1.0)[0])[0] == abi.PIMD_E_UNSUPPORTED
    harm = make_config(wl.systems, None, 0.5, 100.0, 1.0, 1, potential="harmonic", omega=0.01,
                       masses=np.array([1.0, 16.0]), neighbor_skin=1.0)[0]
    assert abi.pimd_workspace_size(harm)[0] == abi.PIMD_E_UNSUPPORTED


def test_g5_workspace_holds_the_moments(lib):
    # G5: per centre 84 floats of moments per (element, eta); G4 instead keeps
    # the in-range slot pairs for its adjoint (16 bits per pair of the 128 slots,
    # and 256 entries of room for the adjoint's look-ahead loads) and ten block
    # counts
    wl = S.workload(2)
    a = abi.pimd_workspace_size(_cfg(wl)[0])[1]
    b = abi.pimd_workspace_size(_cfg(S.with_g5(wl))[0])[1]
    m = wl.model
    moments = wl.bead_atoms * m.n_elements * len(m.ang_eta) * 84 * 4
    pairs = wl.bead_atoms * ((128 * 127 // 2 + 256) * 2 + 10 * 4)
    assert abs((b - a) - (moments - pairs)) <= 4096


@pytest.mark.parametrize("mutate,status", [
    (lambda cfg, k: setattr(cfg, "n_systems", 0), abi.PIMD_E_ARG),
    (lambda cfg, k: setattr(cfg, "dt_fs", 0.0), abi.PIMD_E_ARG),
    (lambda cfg, k: setattr(cfg, "precision", 7), abi.PIMD_E_ARG),
    (lambda cfg, k: setattr(cfg, "potential", 9), abi.PIMD_E_ARG),
    (lambda cfg, k: setattr(cfg, "transform", 5), abi.PIMD_E_ARG),
    (lambda cfg, k: setattr(cfg, "max_neighbors", 100), abi.PIMD_E_ARG),
    (lambda cfg, k: setattr(cfg, "max_neighbors", 1000), abi.PIMD_E_UNSUPPORTED),
    (lambda cfg, k: setattr(cfg, "species", None), abi.PIMD_E_ARG),
    (lambda cfg, k: setattr(cfg, "model", None), abi.PIMD_E_ARG),
    (lambda cfg, k: cfg.n_beads.__setitem__(0, 3), abi.PIMD_E_UNSUPPORTED),     # odd P
    (lambda cfg, k: cfg.n_beads.__setitem__(0, 256), abi.PIMD_E_UNSUPPORTED),   # P > 128
    (lambda cfg, k: cfg.n_atoms.__setitem__(0, 0), abi.PIMD_E_ARG),
    (lambda cfg, k: cfg.temperature_K.__setitem__(0, -1.0), abi.PIMD_E_ARG),
    (lambda cfg, k: cfg.box_A.__setitem__(0, 11.0), abi.PIMD_E_UNSUPPORTED),     # R_c >= L/2
    (lambda cfg, k: cfg.box_A.__setitem__(1, 0.0), abi.PIMD_E_ARG),              # partly zero box
    (lambda cfg, k: cfg.species.__setitem__(0, 5), abi.PIMD_E_ARG),
    (lambda cfg, k: setattr(cfg.model.contents, "n_elements", 0), abi.PIMD_E_UNSUPPORTED),
    (lambda cfg, k: setattr(cfg.model.contents, "n_ang_eta", 3), abi.PIMD_E_UNSUPPORTED),
    (lambda cfg, k: setattr(cfg.model.contents, "angular", 2), abi.PIMD_E_ARG),
    (lambda cfg, k: cfg.model.contents.hidden.__setitem__(0, 40), abi.PIMD_E_UNSUPPORTED),
    (lambda cfg, k: cfg.model.contents.feat_scale.__setitem__(0, 0.0), abi.PIMD_E_ARG),
])
def test_bad_configs_are_rejected_without_a_gpu(lib, mutate, status):
    cfg, keep = _cfg(S.workload(2))
    mutate(cfg, keep)
    st, _ = abi.pimd_workspace_size(cfg)
    assert st == status
    assert abi.pimd_last_error(None)
    st, ctx = abi.pimd_init(cfg, 256, 1 << 30, 0)
    assert st == status and ctx is None


def test_init_rejects_bad_workspace_before_device_work(lib):
    cfg, keep = _cfg(S.workload(1))
    st, n = abi.pimd_workspace_size(cfg)
    assert abi.pimd_init(cfg, 0, n, 0)[0] == abi.PIMD_E_ARG           # NULL workspace
    assert abi.pimd_init(cfg, 4096 + 8, n, 0)[0] == abi.PIMD_E_ARG    # misaligned
    assert abi.pimd_init(cfg, 4096, n - 1, 0)[0] == abi.PIMD_E_OOM     # too small


def test_harmonic_config_needs_omega(lib):
    wl = S.small_workload("fad")
    cfg, keep = make_config(wl.systems, None, 0.5, 100.0, 1.0, 1, potential="harmonic", omega=0.0,
                            masses=wl.model.masses)
    assert abi.pimd_workspace_size(cfg)[0] == abi.PIMD_E_ARG
    cfg, keep = make_config(wl.systems, None, 0.5, 100.0, 1.0, 1, potential="harmonic", omega=0.01,
                            masses=wl.model.masses)
    assert abi.pimd_workspace_size(cfg)[0] == abi.PIMD_OK


def test_null_context_calls_are_argument_errors(lib):
    assert lib.pimd_step(None, 1) == abi.PIMD_E_ARG
    assert lib.pimd_set_state(None, None, None, 0) == abi.PIMD_E_ARG
    assert lib.pimd_energy_forces(None, None, None, None, None) == abi.PIMD_E_ARG
    lib.pimd_destroy(None)


def _md_cfg(wl, **over):
    spec = S.metad_spec(wl)
    for k, v in over.items():
        setattr(spec, k, v)
    return _cfg(wl, metad=spec)


def test_metad_configs_size_the_hill_store(lib):
    for c in (1, 2):
        wl = S.workload(c)
        base = abi.pimd_workspace_size(_cfg(wl)[0])[1]
        st, a = abi.pimd_workspace_size(_md_cfg(wl, max_hills=16)[0])
        st2, b = abi.pimd_workspace_size(_md_cfg(wl, max_hills=4096)[0])
        assert st == st2 == abi.PIMD_OK and base < a < b
        beads = sum(s.n_beads for s in wl.systems)
        assert b - a >= beads * (4096 - 16) * 16


@pytest.mark.parametrize("c,over,status", [
    (1, dict(sigma=0.0), abi.PIMD_E_ARG),
    (1, dict(gamma=1.0), abi.PIMD_E_ARG),
    (1, dict(gamma=float("nan")), abi.PIMD_E_ARG),
    (1, dict(height0=-1.0), abi.PIMD_E_ARG),
    (1, dict(stride=0), abi.PIMD_E_ARG),
    (1, dict(max_hills=0), abi.PIMD_E_ARG),
    (1, dict(atoms=np.array([[0, 10]]), coef=np.array([1.0])), abi.PIMD_E_ARG),  # atom 10 of 10
    (1, dict(atoms=np.array([[3, 3]]), coef=np.array([1.0])), abi.PIMD_E_ARG),
    (2, dict(q_scatter=0.0), abi.PIMD_E_ARG),
    (2, dict(form_factor=np.array([1.0, np.inf])), abi.PIMD_E_ARG),
])
def test_bad_metad_configs_are_rejected_without_a_gpu(lib, c, over, status):
    cfg, keep = _md_cfg(S.workload(c), **over)
    assert abi.pimd_workspace_size(cfg)[0] == status
    assert abi.pimd_last_error(None)


def test_metad_calls_need_a_context(lib):
    assert lib.pimd_bias_forces(None, None, None, None, None) == abi.PIMD_E_ARG
    assert lib.pimd_metad_cv(None, None, None) == abi.PIMD_E_ARG
    assert lib.pimd_metad_set_hills(None, 0, None, None) == abi.PIMD_E_ARG
    assert lib.pimd_metad_fes(None, 0, 0, None, None) == abi.PIMD_E_ARG


def test_static_init_refuses_a_workspace_larger_than_its_array(lib):
    # water 64, P = 32 needs about 130 MiB; the check precedes every HIP call
    cfg, keep = _cfg(S.workload(2))
    assert abi.pimd_workspace_size(cfg)[1] > abi.PIMD_STATIC_WORKSPACE_BYTES
    st, ctx = abi.pimd_init_static(cfg, 0)
    assert st == abi.PIMD_E_CAPACITY and not ctx
    assert "static workspace" in abi.pimd_last_error(None)
    bad, keep2 = _cfg(S.workload(1), neighbor_skin=1.0)
    assert abi.pimd_init_static(bad, 0)[0] == abi.PIMD_E_UNSUPPORTED


def test_thermostat_is_validated(lib):
    wl = S.workload(1)
    assert abi.pimd_workspace_size(_cfg(wl, thermostat="pile-g")[0])[0] == abi.PIMD_OK
    cfg, keep = _cfg(wl)
    cfg.thermostat = 7
    assert abi.pimd_workspace_size(cfg)[0] == abi.PIMD_E_ARG
    # PILE-G thermostats normal modes only
    st = abi.pimd_workspace_size(_cfg(wl, thermostat="pile-g", transform="staging")[0])[0]
    assert st == abi.PIMD_E_UNSUPPORTED
    # its buffers: per integrator unit and per system
    a = abi.pimd_workspace_size(_cfg(wl)[0])[1]
    b = abi.pimd_workspace_size(_cfg(wl, thermostat="pile-g")[0])[1]
    assert b > a


def test_synthetic_weights_are_bfloat16_values_unless_asked_otherwise():
    # the default synthetic networks hold float32 weights with zero low 16 bits
    # (a BF16 MLP then splits only its activations); bf16_weights=False keeps
    # the float32 draws, and rounding moves a weight by at most half a bfloat16 ulp
    wb, wf = S.workload(2).model.weights, S.workload(2, bf16_weights=False).model.weights
    for lb, lf in zip(wb, wf):
        for (Wb, _), (Wf, _) in zip(lb, lf):
            assert Wb.dtype == np.float32 and not np.any(Wb.view(np.uint32) & 0xFFFF)
            assert np.any(Wf.view(np.uint32) & 0xFFFF)
            assert np.all(np.abs(Wb - Wf) <= np.abs(Wf) * 2.0 ** -8)
