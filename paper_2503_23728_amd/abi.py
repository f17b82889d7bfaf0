"""ctypes binding of libpimd.so (include/pimd.h), same names as the C ABI.

Argument marshalling only: every step of the ring-polymer path runs in the
HIP kernels behind these calls.  Loading fails loudly when the library has
not been built (build with paper_2503_23728_amd.build.build()).
"""
import ctypes
import os
import re
from ctypes import POINTER, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpimd.so")
HEADER = os.path.join(HERE, "..", "include", "pimd.h")

PIMD_OK, PIMD_E_ARG, PIMD_E_UNSUPPORTED, PIMD_E_DEVICE, PIMD_E_OOM, PIMD_E_CAPACITY, PIMD_E_NONFINITE, \
    PIMD_E_STATE = range(8)
PIMD_PREC_FP32, PIMD_PREC_BF16_MLP, PIMD_PREC_BF16_PLAIN, PIMD_PREC_FP64_MLP = 0, 1, 2, 3
PIMD_POT_BPNN, PIMD_POT_HARMONIC, PIMD_POT_GFN = 0, 1, 2
PIMD_CV_DISTANCES, PIMD_CV_XRD = 1, 2
PIMD_TRANSFORM_NORMAL_MODES, PIMD_TRANSFORM_STAGING, PIMD_TRANSFORM_PRIMITIVE = 0, 1, 2
PIMD_THERMOSTAT_PILE_L, PIMD_THERMOSTAT_PILE_G = 0, 1


class pimd_bpnn_model(ctypes.Structure):
    _fields_ = [("n_elements", c_int32), ("mass_amu", POINTER(c_double)), ("cutoff_A", c_double),
                ("n_rad", c_int32), ("rad_center_A", POINTER(c_double)), ("rad_eta", POINTER(c_double)),
                ("n_ang_eta", c_int32), ("ang_eta", POINTER(c_double)),
                ("n_hidden", c_int32), ("hidden", c_int32 * 3),
                ("params", POINTER(c_float)), ("feat_shift", POINTER(c_float)), ("feat_scale", POINTER(c_float)),
                ("angular", c_int32)]


class pimd_gfn_model(ctypes.Structure):
    _fields_ = [("n_elements", c_int32), ("mass_amu", POINTER(c_double)), ("cutoff_A", c_double),
                ("n_rad", c_int32), ("rad_center_A", POINTER(c_double)), ("rad_eta", POINTER(c_double)),
                ("width", c_int32), ("n_layers", c_int32), ("params", POINTER(c_float))]


class pimd_metad(ctypes.Structure):
    _fields_ = [("cv", c_int32), ("n_terms", c_int32), ("atoms", POINTER(c_int32)), ("coef", POINTER(c_double)),
                ("q_scatter", c_double), ("form_factor", POINTER(c_double)), ("height0_eV", c_double),
                ("sigma", c_double), ("bias_factor", c_double), ("stride", c_int32), ("max_hills", c_int32)]


class pimd_config(ctypes.Structure):
    _fields_ = [("n_systems", c_int32), ("n_atoms", POINTER(c_int32)), ("n_beads", POINTER(c_int32)),
                ("temperature_K", POINTER(c_double)), ("box_A", POINTER(c_double)), ("species", POINTER(c_int32)),
                ("dt_fs", c_double), ("tau0_fs", c_double), ("pile_lambda", c_double), ("seed", c_uint64),
                ("precision", c_int32), ("potential", c_int32), ("model", POINTER(pimd_bpnn_model)),
                ("harmonic_omega_per_fs", c_double), ("max_neighbors", c_int32),
                ("gfn", POINTER(pimd_gfn_model)), ("metad", POINTER(pimd_metad)), ("transform", c_int32),
                ("neighbor_skin_A", c_double), ("thermostat", c_int32)]


class pimd_tuning(ctypes.Structure):
    _fields_ = [("centre_waves", c_int32), ("centre_grid", c_int32), ("mlp_rows", c_int32),
                ("neighbor_cells", c_int32), ("mlp_waves", c_int32),
                ("force_rows", c_int32), ("centre_lanes", c_int32),
                ("mlp_chain", c_int32)]


class pimd_estimates(ctypes.Structure):
    _fields_ = [(n, c_double) for n in ("V_bar", "K_prim", "K_cv", "E_spring", "K_beads", "T_beads",
                                        "H_conserved", "heat_bath", "V_bias", "P_cv")]


_SIGNATURES = {
    "pimd_workspace_size": (c_int32, [POINTER(pimd_config), POINTER(c_size_t)]),
    "pimd_init": (c_int32, [POINTER(pimd_config), c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "pimd_init_static": (c_int32, [POINTER(pimd_config), c_void_p, POINTER(c_void_p)]),
    "pimd_set_stream": (c_int32, [c_void_p, c_void_p]),
    "pimd_set_state": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64]),
    "pimd_get_state": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_int64)]),
    "pimd_get_heat_bath": (c_int32, [c_void_p, POINTER(c_double)]),
    "pimd_set_heat_bath": (c_int32, [c_void_p, POINTER(c_double)]),
    "pimd_check": (c_int32, [c_void_p]),
    "pimd_energy_forces": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pimd_step": (c_int32, [c_void_p, c_int32]),
    "pimd_estimators": (c_int32, [c_void_p, POINTER(pimd_estimates)]),
    "pimd_inject_noise": (c_int32, [c_void_p, c_void_p]),
    "pimd_bias_forces": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pimd_metad_cv": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    "pimd_metad_hills": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_int32)]),
    "pimd_metad_set_hills": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double)]),
    "pimd_metad_fes": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_double), POINTER(c_double)]),
    "pimd_time_bias": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "pimd_debug_neighbors": (c_int32, [c_void_p, c_int32, POINTER(c_int32), c_int64, POINTER(c_int64)]),
    "pimd_debug_descriptors": (c_int32, [c_void_p, c_void_p]),
    "pimd_debug_copy": (c_int32, [c_void_p, c_int32, c_void_p, c_size_t]),
    "pimd_debug_philox": (c_int32, [c_void_p, c_int64, c_int32, c_int64, c_void_p]),
    "pimd_set_graph": (c_int32, [c_void_p, c_int32]),
    "pimd_get_tuning": (c_int32, [c_void_p, POINTER(pimd_tuning)]),
    "pimd_set_tuning": (c_int32, [c_void_p, POINTER(pimd_tuning)]),
    "pimd_autotune": (c_int32, [c_void_p, c_int32, POINTER(pimd_tuning)]),
    "pimd_profile_stages": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "pimd_time_stages": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "pimd_work_counts": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)]),
    "pimd_neighbor_rebuilds": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64)]),
    "pimd_sizes": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32)]),
    "pimd_last_error": (ctypes.c_char_p, [c_void_p]),
    "pimd_status_str": (ctypes.c_char_p, [c_int32]),
    "pimd_destroy": (None, [c_void_p]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2503_23728_amd.build.build() "
                               "(the ring-polymer path has no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def declared_functions():
    """Function names declared in include/pimd.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pimd_status|const char \*|void)\s*\*?\s*(pimd_\w+)\s*\(", text, re.M)))


class PimdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{lib().pimd_status_str(status).decode()} ({status}): {message}")
        self.status = status


# --- thin wrappers with the C names -------------------------------------------

def pimd_workspace_size(cfg):
    n = c_size_t(0)
    st = lib().pimd_workspace_size(ctypes.byref(cfg), ctypes.byref(n))
    return st, n.value


def pimd_init(cfg, workspace_ptr, ws_bytes, stream_ptr):
    out = c_void_p(0)
    st = lib().pimd_init(ctypes.byref(cfg), c_void_p(workspace_ptr), ws_bytes, c_void_p(stream_ptr),
                         ctypes.byref(out))
    return st, out.value


def pimd_init_static(cfg, stream_ptr):
    out = c_void_p(0)
    st = lib().pimd_init_static(ctypes.byref(cfg), c_void_p(stream_ptr), ctypes.byref(out))
    return st, out.value


PIMD_STATIC_WORKSPACE_BYTES = 64 << 20


def pimd_set_stream(ctx, stream_ptr):
    return lib().pimd_set_stream(c_void_p(ctx), c_void_p(stream_ptr))


def pimd_set_state(ctx, q_ptr, p_ptr, step):
    return lib().pimd_set_state(c_void_p(ctx), c_void_p(q_ptr), c_void_p(p_ptr), step)


def pimd_get_state(ctx, q_ptr, p_ptr, f_ptr):
    step = c_int64(0)
    st = lib().pimd_get_state(c_void_p(ctx), c_void_p(q_ptr), c_void_p(p_ptr), c_void_p(f_ptr), ctypes.byref(step))
    return st, step.value


def pimd_get_heat_bath(ctx, n_systems):
    arr = (c_double * n_systems)()
    st = lib().pimd_get_heat_bath(c_void_p(ctx), arr)
    return st, list(arr)


def pimd_set_heat_bath(ctx, heat):
    arr = (c_double * len(heat))(*[float(h) for h in heat])
    return lib().pimd_set_heat_bath(c_void_p(ctx), arr)


def pimd_check(ctx):
    return lib().pimd_check(c_void_p(ctx))


def pimd_energy_forces(ctx, q_ptr, e_ptr, f_ptr, w_ptr):
    return lib().pimd_energy_forces(c_void_p(ctx), c_void_p(q_ptr), c_void_p(e_ptr), c_void_p(f_ptr),
                                    c_void_p(w_ptr))


def pimd_step(ctx, n):
    return lib().pimd_step(c_void_p(ctx), n)


def pimd_estimators(ctx, n_systems):
    arr = (pimd_estimates * n_systems)()
    st = lib().pimd_estimators(c_void_p(ctx), arr)
    return st, arr


def pimd_inject_noise(ctx, xi_ptr):
    return lib().pimd_inject_noise(c_void_p(ctx), c_void_p(xi_ptr))


def pimd_debug_neighbors(ctx, bead, cap):
    buf = (c_int32 * (2 * max(cap, 1)))()
    count = c_int64(0)
    st = lib().pimd_debug_neighbors(c_void_p(ctx), bead, buf, cap, ctypes.byref(count))
    return st, buf, count.value


def pimd_debug_descriptors(ctx, xhat_ptr):
    return lib().pimd_debug_descriptors(c_void_p(ctx), c_void_p(xhat_ptr))


PIMD_BUF_XHAT, PIMD_BUF_DEDG, PIMD_BUF_SLOTS, PIMD_BUF_NBR, PIMD_BUF_NCOUNT, PIMD_BUF_EATOM = range(6)


def pimd_debug_copy(ctx, buffer, dst_ptr, nbytes):
    return lib().pimd_debug_copy(c_void_p(ctx), buffer, c_void_p(dst_ptr), nbytes)


def pimd_debug_philox(ctx, step, half, n, words_ptr):
    return lib().pimd_debug_philox(c_void_p(ctx), step, half, n, c_void_p(words_ptr))


PIMD_N_STAGES = 7
STAGE_NAMES = ("integrate_pre", "neighbors", "descriptors", "mlp", "adjoint", "forces", "integrate_post")


def pimd_set_graph(ctx, enabled):
    return lib().pimd_set_graph(c_void_p(ctx), 1 if enabled else 0)


def pimd_get_tuning(ctx):
    t = pimd_tuning()
    st = lib().pimd_get_tuning(c_void_p(ctx), ctypes.byref(t))
    return st, t


def pimd_set_tuning(ctx, t):
    return lib().pimd_set_tuning(c_void_p(ctx), ctypes.byref(t))


def pimd_autotune(ctx, n_reps):
    t = pimd_tuning()
    st = lib().pimd_autotune(c_void_p(ctx), n_reps, ctypes.byref(t))
    return st, t


def pimd_profile_stages(ctx, n_reps):
    ms = (c_double * PIMD_N_STAGES)()
    st = lib().pimd_profile_stages(c_void_p(ctx), n_reps, ms)
    return st, list(ms)


PIMD_N_FORCE_STAGES = 5
FORCE_STAGE_NAMES = ("neighbors", "descriptors", "mlp", "adjoint", "forces")


def pimd_time_stages(ctx, n_reps):
    ms = (c_double * PIMD_N_FORCE_STAGES)()
    st = lib().pimd_time_stages(c_void_p(ctx), n_reps, ms)
    return st, list(ms)


def pimd_bias_forces(ctx, q_ptr, f_ptr, cv_ptr, v_ptr):
    return lib().pimd_bias_forces(c_void_p(ctx), c_void_p(q_ptr), c_void_p(f_ptr), c_void_p(cv_ptr),
                                  c_void_p(v_ptr))


def _dptr(a):
    return a.ctypes.data_as(POINTER(c_double)) if a is not None else None


def pimd_metad_cv(ctx, cv_out, v_out):
    """cv_out, v_out: float64 numpy arrays [beads] (or None)."""
    return lib().pimd_metad_cv(c_void_p(ctx), _dptr(cv_out), _dptr(v_out))


def pimd_metad_hills(ctx, centers=None, heights=None):
    n = c_int32(0)
    st = lib().pimd_metad_hills(c_void_p(ctx), _dptr(centers), _dptr(heights), ctypes.byref(n))
    return st, n.value


def pimd_metad_set_hills(ctx, n_hills, centers, heights):
    return lib().pimd_metad_set_hills(c_void_p(ctx), n_hills, _dptr(centers), _dptr(heights))


def pimd_metad_fes(ctx, system, grid, out):
    return lib().pimd_metad_fes(c_void_p(ctx), system, len(grid), _dptr(grid), _dptr(out))


def pimd_time_bias(ctx, n_reps):
    ms = c_double(0.0)
    st = lib().pimd_time_bias(c_void_p(ctx), n_reps, ctypes.byref(ms))
    return st, ms.value


def pimd_work_counts(ctx):
    a, b, c = c_int64(0), c_int64(0), c_int64(0)
    st = lib().pimd_work_counts(c_void_p(ctx), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return st, a.value, b.value, c.value


def pimd_neighbor_rebuilds(ctx):
    n, f = c_int64(0), c_int64(0)
    st = lib().pimd_neighbor_rebuilds(c_void_p(ctx), ctypes.byref(n), ctypes.byref(f))
    return st, n.value, f.value


def pimd_sizes(ctx):
    a, b, c = c_int64(0), c_int64(0), c_int32(0)
    st = lib().pimd_sizes(c_void_p(ctx), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return st, a.value, b.value, c.value


def pimd_last_error(ctx):
    return lib().pimd_last_error(c_void_p(ctx) if ctx else None).decode()


def pimd_status_str(status):
    return lib().pimd_status_str(status).decode()


def pimd_destroy(ctx):
    lib().pimd_destroy(c_void_p(ctx))
