"""Behler-Parrinello potential and its analytic forces in FP64 (oracle side).

Energy of one bead: E = sum_i NN_{Z_i}(xhat_i), xhat_i = (G_i - mu_{Z_i}) / sigma_{Z_i},
G_i the symmetry functions of atom i (bpnn_core.c states them), NN a
per-element tanh MLP.  Forces F = -dE/dq by the chain rule written by hand:
dE/dxhat from the transposed layer chain, dE/dG = dE/dxhat / sigma, then the
descriptor vector-Jacobian product per neighbour slot from the C core.  The
energy model of the paper obtains forces this way, by differentiating the
predicted energy with respect to the coordinates (Sec. 2.2).

Virial: W_ab = -sum_i sum_{j in N(i)} d_ij,a dE_i/dd_ij,b, which equals
-dE/deps_ab under the affine strain q -> (1+eps) q, L -> (1+eps) L.
"""
import ctypes
import os

import numpy as np

from . import build as _build
from . import neighbors

_lib = None


def _core():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        common = [ctypes.c_int, P(ctypes.c_double), P(ctypes.c_int32), P(ctypes.c_double), ctypes.c_int,
                  ctypes.c_int, ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double),
                  ctypes.c_int, P(ctypes.c_double), ctypes.c_double,
                  ctypes.c_int, P(ctypes.c_int32), P(ctypes.c_int64), P(ctypes.c_int32)]
        _lib.oracle_descriptors.argtypes = common + [P(ctypes.c_double), P(ctypes.c_int64), ctypes.c_int]
        _lib.oracle_descriptors.restype = None
        _lib.oracle_descriptor_vjp.argtypes = common + [P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int]
        _lib.oracle_descriptor_vjp.restype = None
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class _Call:
    """Holds contiguous arrays alive for one C call."""

    def __init__(self, model, q, species, box, centers, start, idx):
        self.q = np.ascontiguousarray(q, dtype=np.float64)
        self.species = np.ascontiguousarray(species, dtype=np.int32)
        self.box = np.ascontiguousarray(box, dtype=np.float64)
        self.periodic = int(np.any(self.box > 0))
        self.rc_ = np.ascontiguousarray(model.rad_center, dtype=np.float64)
        self.re_ = np.ascontiguousarray(model.rad_eta, dtype=np.float64)
        self.ae_ = np.ascontiguousarray(model.ang_eta, dtype=np.float64)
        self.centers = np.ascontiguousarray(centers, dtype=np.int32)
        self.start = np.ascontiguousarray(start, dtype=np.int64)
        self.idx = np.ascontiguousarray(idx, dtype=np.int32)
        self.model = model

    def args(self):
        m = self.model
        return [len(self.q), _ptr(self.q, ctypes.c_double), _ptr(self.species, ctypes.c_int32),
                _ptr(self.box, ctypes.c_double), self.periodic,
                m.n_elements, m.n_rad, _ptr(self.rc_, ctypes.c_double), _ptr(self.re_, ctypes.c_double),
                len(m.ang_eta), _ptr(self.ae_, ctypes.c_double), float(m.cutoff),
                len(self.centers), _ptr(self.centers, ctypes.c_int32), _ptr(self.start, ctypes.c_int64),
                _ptr(self.idx, ctypes.c_int32)]


def _angular(model):
    """0: G4 angular functions (with the r_jk factors), 1: G5 (without)."""
    kind = getattr(model, "angular", "g4")
    if kind not in ("g4", "g5"):
        raise ValueError(f"unknown angular form {kind!r}")
    return int(kind == "g5")


def descriptors(model, q, species, box, centers, start, idx, with_counts=False):
    """Raw symmetry functions G[len(centers), D] (before normalisation).
    start/idx: CSR neighbour lists of the centres (one row per centre)."""
    call = _Call(model, q, species, box, centers, start, idx)
    G = np.zeros((len(call.centers), model.n_features))
    counts = np.zeros((len(call.centers), 2), dtype=np.int64)
    _core().oracle_descriptors(*call.args(), _ptr(G, ctypes.c_double), _ptr(counts, ctypes.c_int64),
                               _angular(model))
    return (G, counts) if with_counts else G


def descriptor_vjp(model, q, species, box, centers, start, idx, dEdG):
    """Slot vectors v[slot, 3] = dE/dd_{i,j} for every CSR slot."""
    call = _Call(model, q, species, box, centers, start, idx)
    g = np.ascontiguousarray(dEdG, dtype=np.float64)
    v = np.zeros((len(call.idx), 3))
    _core().oracle_descriptor_vjp(*call.args(), _ptr(g, ctypes.c_double), _ptr(v, ctypes.c_double),
                                  _angular(model))
    return v


def normalise(model, G, species_of_centres):
    mu = model.feat_shift.astype(np.float64)[species_of_centres]
    sd = model.feat_scale.astype(np.float64)[species_of_centres]
    return (G - mu) / sd


def mlp_energy_grad(model, species_of_centres, xhat, bf16=False):
    """Per-atom energies E_i = NN_{Z_i}(xhat_i) and dE_i/dxhat_i.

    Forward: h_0 = xhat, h_l = tanh(W_l h_{l-1} + b_l), E = w_out . h_L + b_out.
    Input gradient by the transposed chain:
      g_L = w_out * (1 - h_L^2), g_{l-1} = (W_l^T g_l) * (1 - h_{l-1}^2), dE/dxhat = W_1^T g_1.
    bf16=True rounds the operands of the layer products (inputs,
    activations, upstream gradients and weights) to bfloat16 before each
    product and accumulates in FP64 (the energy readout stays unrounded); it
    mirrors a BF16-operand / wide-accumulate GEMM and is for diagnosis only.
    """
    rnd = _round_bf16 if bf16 else (lambda a: a)
    n, D = xhat.shape
    E = np.zeros(n)
    dx = np.zeros((n, D))
    for e, layers in enumerate(model.weights):
        sel = np.nonzero(species_of_centres == e)[0]
        if len(sel) == 0:
            continue
        hs = [xhat[sel]]
        for W, b in layers[:-1]:
            hs.append(np.tanh(rnd(hs[-1]) @ rnd(W.astype(np.float64)).T + b.astype(np.float64)))
        Wo, bo = layers[-1]
        wo = Wo.astype(np.float64)[0]
        E[sel] = hs[-1] @ wo + float(bo[0])
        g = wo[None, :] * (1.0 - hs[-1] ** 2)
        for l in range(len(layers) - 2, -1, -1):
            up = rnd(g) @ rnd(layers[l][0].astype(np.float64))
            if l == 0:
                dx[sel] = up
            else:
                g = up * (1.0 - hs[l] ** 2)
    return E, dx


def _round_bf16(a):
    """Round float64 values to the nearest bfloat16 (ties to even), via float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bead_neighbors(model, q32_bead, box):
    return neighbors.brute_force_fp32(q32_bead, box, model.cutoff)


def bead_energy_forces(model, q32_bead, species, box, bf16=False, return_parts=False):
    """Energy (eV), forces [N,3] (eV/A) and virial [3,3] (eV) of one bead.

    Neighbour membership comes from the float32 positions (neighbors module);
    everything else is FP64 on float64(q32)."""
    q32_bead = np.asarray(q32_bead, dtype=np.float32)
    q = q32_bead.astype(np.float64)
    n = len(q)
    start, idx = bead_neighbors(model, q32_bead, box)
    centres = np.arange(n, dtype=np.int32)
    G = descriptors(model, q, species, box, centres, start, idx)
    xhat = normalise(model, G, species)
    Ei, dx = mlp_energy_grad(model, species, xhat, bf16=bf16)
    dEdG = dx / model.feat_scale.astype(np.float64)[species]
    v = descriptor_vjp(model, q, species, box, centres, start, idx, dEdG)
    owner = np.repeat(np.arange(n), np.diff(start))
    grad = np.zeros((n, 3))
    np.add.at(grad, idx, v)
    np.add.at(grad, owner, -v)
    d = q[idx] - q[owner]
    if np.any(np.asarray(box) > 0):
        d = d - box * np.round(d / box)
    W = -np.einsum("sa,sb->ab", d, v)
    if return_parts:
        return Ei.sum(), -grad, W, dict(G=G, xhat=xhat, Ei=Ei, dEdG=dEdG, start=start, idx=idx, v=v)
    return Ei.sum(), -grad, W


def energy_forces(wl, q32, bf16=False):
    """All beads of all systems of a workload: E[sum P_s], F[sum P_s N_s, 3], W[sum P_s, 3, 3]."""
    q32 = np.asarray(q32, dtype=np.float32).reshape(-1, 3)
    Es, Fs, Ws = [], [], []
    off = 0
    for s in wl.systems:
        for _k in range(s.n_beads):
            E, F, W = bead_energy_forces(wl.model, q32[off:off + s.n_atoms], s.species, s.box, bf16=bf16)
            Es.append(E)
            Fs.append(F)
            Ws.append(W)
            off += s.n_atoms
    return np.array(Es), np.concatenate(Fs), np.array(Ws)


def atom_forces_sampled(model, q32_bead, species, box, atoms):
    """Forces on selected atoms of one bead, computed from the neighbourhood
    only: F_a needs dE_c/dq_a for c = a and every c with a in N(c).  The
    neighbour lists are the full-bead float32 sets."""
    q32_bead = np.asarray(q32_bead, dtype=np.float32)
    q = q32_bead.astype(np.float64)
    start, idx = bead_neighbors(model, q32_bead, box)
    out = np.zeros((len(atoms), 3))
    for t, a in enumerate(atoms):
        centres = np.concatenate([[a], idx[start[a]:start[a + 1]]]).astype(np.int32)
        cs = np.zeros(len(centres) + 1, dtype=np.int64)
        rows = [idx[start[c]:start[c + 1]] for c in centres]
        np.cumsum([len(r) for r in rows], out=cs[1:])
        cidx = np.concatenate(rows).astype(np.int32)
        G = descriptors(model, q, species, box, centres, cs, cidx)
        sp = species[centres]
        xhat = normalise(model, G, sp)
        _, dx = mlp_energy_grad(model, sp, xhat)
        dEdG = dx / model.feat_scale.astype(np.float64)[sp]
        v = descriptor_vjp(model, q, species, box, centres, cs, cidx, dEdG)
        owner = np.repeat(centres, np.diff(cs))
        g = v[cidx == a].sum(axis=0) - v[owner == a].sum(axis=0)
        out[t] = -g
    return out


def atom_descriptors_sampled(model, q32_bead, species, box, atoms):
    """Normalised descriptors of selected atoms of one bead."""
    q32_bead = np.asarray(q32_bead, dtype=np.float32)
    start, idx = bead_neighbors(model, q32_bead, box)
    atoms = np.asarray(atoms, dtype=np.int32)
    cs = np.zeros(len(atoms) + 1, dtype=np.int64)
    rows = [idx[start[c]:start[c + 1]] for c in atoms]
    np.cumsum([len(r) for r in rows], out=cs[1:])
    cidx = np.concatenate(rows).astype(np.int32)
    G = descriptors(model, q32_bead.astype(np.float64), species, box, atoms, cs, cidx)
    return normalise(model, G, species[atoms])
