"""Torch-facing wrapper of the ring-polymer library.

PyTorch provides the device memory (the workspace and the state tensors)
and the stream; every computation runs in libpimd.so.

    eng = Pimd.from_workload(wl, device="cuda:0", precision="bf16")
    eng.set_state(q, p)
    eng.step(100)
    est = eng.estimators()

`PimdEnergy` is the autograd view: forward gives the per-bead energies,
backward returns -gE[bead] * F from the adjoint kernels.
"""
import ctypes

import numpy as np
import torch

from . import abi, tuning


def _check(st, ctx=None):
    if st != abi.PIMD_OK:
        raise abi.PimdError(st, abi.pimd_last_error(ctx))


def _ptr(t):
    return 0 if t is None else t.data_ptr()


def pack_params(model):
    """Concatenate per element: each layer's W [out][in] row-major, then b."""
    parts = []
    for layers in model.weights:
        for W, b in layers:
            parts.append(np.ascontiguousarray(W, dtype=np.float32).ravel())
            parts.append(np.ascontiguousarray(b, dtype=np.float32).ravel())
    return np.concatenate(parts).astype(np.float32)


class _Keep:
    """Host arrays that must outlive the config structs during pimd_init."""

    def __init__(self):
        self.items = []

    def arr(self, a, dtype, ctype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.items.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctype))


def pack_gfn_params(head):
    """The direct-force head's weights in the order include/pimd.h gives."""
    parts = [head.node_embed, head.pair_embed, head.edge_in]
    for msg, node, edge in head.layers:
        for W1, b1, W2, b2 in (msg, node, edge):
            parts += [W1, b1, W2, b2]
    W1, b1, w2, b2 = head.force
    parts += [W1, b1, w2, np.array([b2])]
    return np.concatenate([np.ascontiguousarray(a, dtype=np.float32).ravel() for a in parts])


def make_metad(spec, keep):
    """pimd_metad from a synthetic.MetadSpec (cv "distances" or "xrd")."""
    md = abi.pimd_metad()
    if spec.cv == "distances":
        md.cv = abi.PIMD_CV_DISTANCES
        if np.asarray(spec.atoms).size != 2 * len(spec.coef):
            raise ValueError("distance CV: atoms must hold two indices per coefficient")
        md.n_terms = len(spec.coef)
        md.atoms = keep.arr(np.asarray(spec.atoms).reshape(-1), np.int32, ctypes.c_int32)
        md.coef = keep.arr(spec.coef, np.float64, ctypes.c_double)
    elif spec.cv == "xrd":
        md.cv = abi.PIMD_CV_XRD
        md.q_scatter = float(spec.q_scatter)
        md.form_factor = keep.arr(spec.form_factor, np.float64, ctypes.c_double)
    else:
        raise ValueError(f"unknown collective variable {spec.cv!r}")
    md.height0_eV = float(spec.height0)
    md.sigma = float(spec.sigma)
    md.bias_factor = float(spec.gamma)
    md.stride = int(spec.stride)
    md.max_hills = int(spec.max_hills)
    keep.items.append(md)
    return md


ANGULAR = {"g4": 0, "g5": 1}     # PIMD_ANGULAR_G4, PIMD_ANGULAR_G5


def make_config(systems, model, dt, tau0, pile_lambda, seed, precision="fp32", potential="bpnn",
                omega=0.0, max_neighbors=0, masses=None, metad=None, transform="normal-modes", neighbor_skin=0.0,
                thermostat="pile-l"):
    """Build the pimd_config (and the storage it points into).

    systems: sequence with n_atoms, n_beads, temperature, box, species.
    model: a synthetic.Model (BPNN), a synthetic.GfnModel (direct-force head,
    potential "gfn"), or None with `masses` (harmonic)."""
    keep = _Keep()
    m = abi.pimd_bpnn_model()
    g = None
    if potential == "gfn":
        g = abi.pimd_gfn_model()
        g.n_elements = model.n_elements
        g.mass_amu = keep.arr(model.masses, np.float64, ctypes.c_double)
        g.cutoff_A = float(model.cutoff)
        g.n_rad = model.n_rad
        g.rad_center_A = keep.arr(model.rad_center, np.float64, ctypes.c_double)
        g.rad_eta = keep.arr(model.rad_eta, np.float64, ctypes.c_double)
        g.width = model.width
        g.n_layers = model.n_layers
        g.params = keep.arr(pack_gfn_params(model), np.float32, ctypes.c_float)
        keep.items.append(g)
    elif model is not None:
        m.n_elements = model.n_elements
        m.mass_amu = keep.arr(model.masses, np.float64, ctypes.c_double)
        m.cutoff_A = float(model.cutoff)
        m.n_rad = model.n_rad
        m.rad_center_A = keep.arr(model.rad_center, np.float64, ctypes.c_double)
        m.rad_eta = keep.arr(model.rad_eta, np.float64, ctypes.c_double)
        m.n_ang_eta = len(model.ang_eta)
        m.ang_eta = keep.arr(model.ang_eta, np.float64, ctypes.c_double)
        m.n_hidden = len(model.hidden)
        for l, h in enumerate(model.hidden):
            m.hidden[l] = h
        m.params = keep.arr(pack_params(model), np.float32, ctypes.c_float)
        m.feat_shift = keep.arr(model.feat_shift, np.float32, ctypes.c_float)
        m.feat_scale = keep.arr(model.feat_scale, np.float32, ctypes.c_float)
        angular = getattr(model, "angular", "g4")
        if angular not in ANGULAR:
            raise ValueError(f"angular must be one of {sorted(ANGULAR)}")
        m.angular = ANGULAR[angular]
    else:
        m.n_elements = len(masses)
        m.mass_amu = keep.arr(masses, np.float64, ctypes.c_double)
    keep.items.append(m)
    cfg = abi.pimd_config()
    cfg.n_systems = len(systems)
    cfg.n_atoms = keep.arr([s.n_atoms for s in systems], np.int32, ctypes.c_int32)
    cfg.n_beads = keep.arr([s.n_beads for s in systems], np.int32, ctypes.c_int32)
    cfg.temperature_K = keep.arr([s.temperature for s in systems], np.float64, ctypes.c_double)
    cfg.box_A = keep.arr(np.concatenate([np.asarray(s.box, dtype=np.float64) for s in systems]), np.float64,
                         ctypes.c_double)
    cfg.species = keep.arr(np.concatenate([np.asarray(s.species) for s in systems]), np.int32, ctypes.c_int32)
    cfg.dt_fs = dt
    cfg.tau0_fs = tau0
    cfg.pile_lambda = pile_lambda
    cfg.seed = seed
    cfg.precision = {"fp32": abi.PIMD_PREC_FP32, "bf16": abi.PIMD_PREC_BF16_MLP,
                     "bf16-plain": abi.PIMD_PREC_BF16_PLAIN, "fp64-mlp": abi.PIMD_PREC_FP64_MLP}[precision]
    cfg.potential = {"bpnn": abi.PIMD_POT_BPNN, "harmonic": abi.PIMD_POT_HARMONIC,
                     "gfn": abi.PIMD_POT_GFN}[potential]
    cfg.model = ctypes.pointer(m)
    cfg.gfn = ctypes.pointer(g) if g is not None else None
    cfg.harmonic_omega_per_fs = omega
    cfg.max_neighbors = max_neighbors
    cfg.metad = ctypes.pointer(make_metad(metad, keep)) if metad is not None else None
    cfg.transform = {"normal-modes": abi.PIMD_TRANSFORM_NORMAL_MODES, "staging": abi.PIMD_TRANSFORM_STAGING,
                     "primitive": abi.PIMD_TRANSFORM_PRIMITIVE}[transform]
    cfg.neighbor_skin_A = float(neighbor_skin)
    cfg.thermostat = {"pile-l": abi.PIMD_THERMOSTAT_PILE_L, "pile-g": abi.PIMD_THERMOSTAT_PILE_G}[thermostat]
    return cfg, keep


MAX_NEIGHBORS = 256          # the library's largest slot count per atom


def grown_slots(k):
    """Slot count after a neighbour overflow at k slots: 1.5 k rounded up to a
    multiple of 16, at most MAX_NEIGHBORS; None when k is already the most."""
    k = k or 128
    if k >= MAX_NEIGHBORS:
        return None
    return min(MAX_NEIGHBORS, (3 * k // 2 + 15) // 16 * 16)


class Pimd:
    """One library context: state, workspace and stream on one device.

    static_workspace=True builds the context with pimd_init_static on the
    library's own per-device array (no device allocation at all; small
    systems only, one such context per device at a time).

    regrow=True: when a synchronising call reports that an atom had more
    neighbours than the slots per atom (PIMD_E_CAPACITY), the context is built
    again with more slots (grown_slots), the state the library froze at (the
    last step completed before the overflow, with its heat bath, hills and
    launch shape) is put back, the steps asked for since are replayed, and the
    call is made again."""

    def __init__(self, systems, model, dt, tau0, pile_lambda, seed, precision="fp32", potential="bpnn",
                 omega=0.0, max_neighbors=0, masses=None, device="cuda:0", stream=None, metad=None,
                 transform="normal-modes", neighbor_skin=0.0, regrow=True, static_workspace=False,
                 thermostat="pile-l"):
        self.device = torch.device(device)
        self.metad = metad
        self.systems = list(systems)
        self.model, self.precision, self.max_neighbors = model, precision, max_neighbors
        self.neighbor_skin = float(neighbor_skin)
        self.regrow = regrow
        self.regrowths = 0
        self.static_workspace = bool(static_workspace)
        self._cfg_args = (dt, tau0, pile_lambda, seed, precision, potential, omega, masses, metad, transform,
                          neighbor_skin, thermostat)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = None
        self._target_step = 0          # steps the caller has asked for, counted from set_state
        self._use_graph = True
        self._open(max_neighbors)
        bead_of_row = []
        b0 = 0
        for s in self.systems:
            bead_of_row.append(b0 + np.repeat(np.arange(s.n_beads), s.n_atoms))
            b0 += s.n_beads
        self.bead_of_row = torch.as_tensor(np.concatenate(bead_of_row), device=self.device, dtype=torch.long)

    def _open(self, max_neighbors):
        dt, tau0, lam, seed, precision, potential, omega, masses, metad, transform, skin, thermostat = self._cfg_args
        self.max_neighbors = max_neighbors
        self.cfg, self._keep = make_config(self.systems, self.model, dt, tau0, lam, seed, precision, potential,
                                           omega, max_neighbors, masses, metad, transform, skin, thermostat)
        if self.static_workspace:
            # the library's own per-device array: no device allocation at all
            self.workspace = None
            with torch.cuda.device(self.device):
                st, ctx = abi.pimd_init_static(self.cfg, self.stream.cuda_stream)
            _check(st)
        else:
            st, nbytes = abi.pimd_workspace_size(self.cfg)
            _check(st)
            self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            if self.workspace.data_ptr() % 256:
                raise RuntimeError("torch returned a workspace that is not 256-byte aligned")
            st, ctx = abi.pimd_init(self.cfg, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
            _check(st)
        self.ctx = ctx
        st, self.B, self.n_beads, self.D = abi.pimd_sizes(ctx)
        _check(st, ctx)

    def _grow(self):
        """Rebuild with more neighbour slots after an overflow; False when no
        larger slot count exists."""
        k = grown_slots(self.max_neighbors)
        if k is None:
            return False
        q = torch.empty(self.B, 3, device=self.device)
        p = torch.empty_like(q)
        st, step = abi.pimd_get_state(self.ctx, q.data_ptr(), p.data_ptr(), 0)
        state_set = st != abi.PIMD_E_STATE
        if state_set:
            _check(st, self.ctx)
            st, heat = abi.pimd_get_heat_bath(self.ctx, len(self.systems))
            _check(st, self.ctx)
        hills = self.metad_hills() if self.metad is not None else None
        shape = self.get_tuning()
        abi.pimd_destroy(self.ctx)
        self.ctx = None
        self._open(k)
        self.regrowths += 1
        self.set_tuning(**shape)
        self.set_graph(self._use_graph)
        if hills is not None and hills[0].shape[1]:
            self.metad_set_hills(*hills)
        if state_set:
            target = self._target_step
            _check(abi.pimd_set_state(self.ctx, q.data_ptr(), p.data_ptr(), int(step)), self.ctx)
            _check(abi.pimd_set_heat_bath(self.ctx, heat), self.ctx)
            self._target_step = target
            if target > step:
                _check(abi.pimd_step(self.ctx, int(target - step)), self.ctx)
        return True

    def _sync(self, call):
        """Run a synchronising library call (a function of the context); regrow
        and run it again while it reports a neighbour overflow."""
        while True:
            st = call(self.ctx)
            if (st == abi.PIMD_E_CAPACITY and self.regrow and "max_neighbors" in abi.pimd_last_error(self.ctx)
                    and self._grow()):
                continue
            _check(st, self.ctx)
            return
        bead_of_row = []
        b0 = 0
        for s in self.systems:
            bead_of_row.append(b0 + np.repeat(np.arange(s.n_beads), s.n_atoms))
            b0 += s.n_beads
        self.bead_of_row = torch.as_tensor(np.concatenate(bead_of_row), device=self.device, dtype=torch.long)

    @classmethod
    def from_workload(cls, wl, **kw):
        """A context for a synthetic workload; a workload whose model is the
        direct-force head selects potential "gfn"."""
        if type(wl.model).__name__ == "GfnModel":
            kw.setdefault("potential", "gfn")
        return cls(wl.systems, wl.model, wl.dt, wl.tau0, wl.pile_lambda, wl.philox_seed, **kw)

    def close(self):
        """Destroy the library context (synchronises); the workspace is freed with the object."""
        if getattr(self, "ctx", None):
            abi.pimd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass     # interpreter shutdown: the binding may already be gone

    def _vec(self, x, shape):
        t = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        if tuple(t.shape) != shape:
            t = t.reshape(shape)
        return t

    def set_state(self, q, p, step=0, heat_bath=None):
        """Positions, momenta and step counter; heat_bath (one value per system,
        from get_heat_bath) restores the thermostat's account of a checkpoint,
        else it starts at zero."""
        q = self._vec(q, (self.B, 3))
        p = self._vec(p, (self.B, 3))
        _check(abi.pimd_set_state(self.ctx, q.data_ptr(), p.data_ptr(), int(step)), self.ctx)
        if heat_bath is not None:
            _check(abi.pimd_set_heat_bath(self.ctx, list(heat_bath)), self.ctx)
        self._target_step = int(step)

    def get_state(self, forces=True):
        q = torch.empty(self.B, 3, device=self.device)
        p = torch.empty_like(q)
        F = torch.empty_like(q) if forces else None
        out = {}

        def call(ctx):
            st, out["step"] = abi.pimd_get_state(ctx, q.data_ptr(), p.data_ptr(), _ptr(F))
            return st
        self._sync(call)
        return q, p, F, out["step"]

    def get_heat_bath(self):
        st, heat = abi.pimd_get_heat_bath(self.ctx, len(self.systems))
        _check(st, self.ctx)
        return heat

    def check(self):
        """Wait for the enqueued work and raise on a latched device fault (after
        regrowing and replaying, for a neighbour overflow with regrow=True)."""
        self._sync(abi.pimd_check)

    def energy_forces(self, q, forces=True, virial=False, check=True):
        """Energies [beads], forces [B, 3] and virials [beads, 3, 3] at q.  With
        check=True the call waits for the kernels and raises on a device fault
        (a neighbour overflow regrows the context and evaluates again)."""
        q = self._vec(q, (self.B, 3))
        E = torch.empty(self.n_beads, device=self.device)
        F = torch.empty(self.B, 3, device=self.device) if forces else None
        W = torch.empty(self.n_beads, 3, 3, device=self.device) if virial else None

        def call(ctx):
            st = abi.pimd_energy_forces(ctx, q.data_ptr(), E.data_ptr(), _ptr(F), _ptr(W))
            return abi.pimd_check(ctx) if st == abi.PIMD_OK and check else st
        self._sync(call)
        return E, F, W

    def step(self, n=1):
        _check(abi.pimd_step(self.ctx, int(n)), self.ctx)
        self._target_step += int(n)

    def estimators(self):
        out = {}

        def call(ctx):
            st, out["arr"] = abi.pimd_estimators(ctx, len(self.systems))
            return st
        self._sync(call)
        return [{f: getattr(a, f) for f, _ in abi.pimd_estimates._fields_} for a in out["arr"]]

    def inject_noise(self, xi):
        xi = self._vec(xi, (2, self.B, 3))
        _check(abi.pimd_inject_noise(self.ctx, xi.data_ptr()), self.ctx)
        self._xi_keep = xi

    def set_graph(self, enabled):
        _check(abi.pimd_set_graph(self.ctx, enabled), self.ctx)
        self._use_graph = bool(enabled)

    def get_tuning(self):
        """The launch shape of the force kernels: {centre_waves, centre_grid, mlp_rows, neighbor_cells}."""
        st, t = abi.pimd_get_tuning(self.ctx)
        _check(st, self.ctx)
        return {f: getattr(t, f) for f in tuning.FIELDS}

    def set_tuning(self, **shape):
        cur = self.get_tuning()
        cur.update(shape)
        t = abi.pimd_tuning(*(cur[f] for f in tuning.FIELDS))
        _check(abi.pimd_set_tuning(self.ctx, t), self.ctx)

    def tuning_key(self):
        props = torch.cuda.get_device_properties(self.device)
        arch = getattr(props, "gcnArchName", props.name)
        return tuning.config_key(arch, props.multi_processor_count, self.systems, self.model, self.precision,
                                 self.max_neighbors, self.neighbor_skin)

    def autotune(self, n_reps=5, cache=True):
        """Pick the fastest launch shape for this batch (needs the state set).

        With cache=True a shape stored for the same GPU and configuration is
        applied without timing; otherwise pimd_autotune sweeps the candidates
        on the current positions and the winner is stored.  Returns the shape
        and whether it came from the cache."""
        key = self.tuning_key()
        if cache:
            hit = tuning.load(key)
            if hit is not None:
                self.set_tuning(**hit)
                return hit, True
        st, t = abi.pimd_autotune(self.ctx, int(n_reps))
        _check(st, self.ctx)
        shape = {f: getattr(t, f) for f in tuning.FIELDS}
        if cache:
            tuning.store(key, shape)
        return shape, False

    def profile_stages(self, n_reps):
        """Mean ms per step of each stage (abi.STAGE_NAMES), HIP events on the context stream."""
        st, ms = abi.pimd_profile_stages(self.ctx, int(n_reps))
        _check(st, self.ctx)
        return dict(zip(abi.STAGE_NAMES, ms))

    def time_stages(self, n_reps):
        """Mean ms of one run of each force stage (abi.FORCE_STAGE_NAMES), each stage
        enqueued n_reps times back to back between HIP events; the state does not move."""
        st, ms = abi.pimd_time_stages(self.ctx, int(n_reps))
        _check(st, self.ctx)
        return dict(zip(abi.FORCE_STAGE_NAMES, ms))

    def neighbor_rebuilds(self):
        """(builds of the shared centroid lists, force evaluations that scanned whole
        beads because a ring was wider than the skin), contexts with a skin."""
        st, n, f = abi.pimd_neighbor_rebuilds(self.ctx)
        _check(st, self.ctx)
        return n, f

    def work_counts(self):
        """(pairs, triplets, triplets with r_jk < cutoff) of the last force evaluation."""
        st, a, b, c = abi.pimd_work_counts(self.ctx)
        _check(st, self.ctx)
        return a, b, c

    # ---- well-tempered metadynamics (contexts built with metad=MetadSpec)
    def bias_forces(self, q, forces=True):
        """(bias forces [B, 3] or None, CV [beads], bias energy [beads]) at q
        with the current hills; no deposition."""
        q = self._vec(q, (self.B, 3))
        F = torch.empty(self.B, 3, device=self.device) if forces else None
        cv = torch.empty(self.n_beads, dtype=torch.float64, device=self.device)
        v = torch.empty_like(cv)
        _check(abi.pimd_bias_forces(self.ctx, q.data_ptr(), _ptr(F), cv.data_ptr(), v.data_ptr()), self.ctx)
        return F, cv, v

    def metad_cv(self):
        """(CV, bias energy) per bead at the current state, numpy float64."""
        cv, v = np.zeros(self.n_beads), np.zeros(self.n_beads)
        _check(abi.pimd_metad_cv(self.ctx, cv, v), self.ctx)
        return cv, v

    def metad_hills(self):
        """(centers, heights) [beads, n_hills] numpy float64."""
        st, n = abi.pimd_metad_hills(self.ctx)
        _check(st, self.ctx)
        c, h = np.zeros((self.n_beads, n)), np.zeros((self.n_beads, n))
        st, n2 = abi.pimd_metad_hills(self.ctx, c, h)
        _check(st, self.ctx)
        return c[:, :n2], h[:, :n2]

    def metad_set_hills(self, centers, heights):
        c = np.ascontiguousarray(centers, dtype=np.float64).reshape(self.n_beads, -1)
        h = np.ascontiguousarray(heights, dtype=np.float64).reshape(self.n_beads, -1)
        if c.shape != h.shape:
            raise ValueError("centers and heights differ in shape")
        _check(abi.pimd_metad_set_hills(self.ctx, c.shape[1], c, h), self.ctx)

    def metad_fes(self, system, grid):
        """Quantum free-energy surface (eV) of one system on a grid."""
        g = np.ascontiguousarray(grid, dtype=np.float64)
        out = np.zeros_like(g)
        _check(abi.pimd_metad_fes(self.ctx, int(system), g, out), self.ctx)
        return out

    def time_bias(self, n_reps):
        """Mean ms of one bias pass (CV kernels, bias, bias forces) at the current positions."""
        st, ms = abi.pimd_time_bias(self.ctx, int(n_reps))
        _check(st, self.ctx)
        return ms

    def debug_neighbors(self, bead):
        cap = 1 << 22
        st, buf, count = abi.pimd_debug_neighbors(self.ctx, bead, cap)
        _check(st, self.ctx)
        return np.ctypeslib.as_array(buf)[: 2 * count].reshape(-1, 2).copy()

    def debug_descriptors(self):
        x = torch.empty(self.B, self.D, device=self.device)
        _check(abi.pimd_debug_descriptors(self.ctx, x.data_ptr()), self.ctx)
        return x

    def debug_buffer(self, name):
        """Internal buffer of the last force evaluation: 'xhat', 'dEdG', 'slots', 'nbr', 'ncount', 'eatom'."""
        K = self.cfg.max_neighbors or 128
        spec = {"xhat": (abi.PIMD_BUF_XHAT, (self.B, self.D), torch.float32),
                "dEdG": (abi.PIMD_BUF_DEDG, (self.B, self.D), torch.float32),
                "slots": (abi.PIMD_BUF_SLOTS, (self.B, K, 4), torch.float32),
                "nbr": (abi.PIMD_BUF_NBR, (self.B, K), torch.int32),
                "ncount": (abi.PIMD_BUF_NCOUNT, (self.B,), torch.int32),
                "eatom": (abi.PIMD_BUF_EATOM, (self.B,), torch.float32)}[name]
        t = torch.empty(spec[1], dtype=spec[2], device=self.device)
        _check(abi.pimd_debug_copy(self.ctx, spec[0], t.data_ptr(), t.numel() * t.element_size()), self.ctx)
        return t

    def debug_philox(self, step, half, n):
        w = torch.empty(n, 4, dtype=torch.int32, device=self.device)
        _check(abi.pimd_debug_philox(self.ctx, int(step), int(half), int(n), w.data_ptr()), self.ctx)
        return w


class PimdEnergy(torch.autograd.Function):
    """E_bead = PimdEnergy.apply(q, engine): per-bead potential energies;
    the backward pass runs the adjoint (descriptor recomputation) kernels."""

    @staticmethod
    def forward(ctx, q, engine):
        E, _, _ = engine.energy_forces(q.detach(), forces=False)
        ctx.save_for_backward(q.detach())
        ctx.engine = engine
        return E

    @staticmethod
    def backward(ctx, gE):
        (q,) = ctx.saved_tensors
        eng = ctx.engine
        _, F, _ = eng.energy_forces(q, forces=True)
        return -gE[eng.bead_of_row][:, None] * F, None
