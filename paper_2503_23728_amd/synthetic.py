"""Seeded synthetic workloads for ring-polymer MD with a symmetry-function
neural potential.

This module only draws inputs: geometries, element tables, descriptor grids,
random network weights and initial momenta.  It holds none of the method's
arithmetic (no neighbour search, descriptors, network evaluation, normal
modes or thermostat), so both the FP64 CPU oracle and the GPU library can be
fed from it without sharing any computation.

The systems mirror the paper's two case studies by shape only: the formic
acid dimer (Sec. 3.1) and liquid water / ice-Ih (Sec. 3.2, Table S3), with
the cutoff of Tables S1/S2 (0.6 nm) and the PIMD settings of Table S3 /
Sec. S1.  The potential family is the Behler-Parrinello descriptor network
the introduction cites; its grid and widths are hyperparameters stated here.

Units: Angstrom, fs, amu, eV.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
import math

import numpy as np

# Element data: IUPAC conventional atomic weights.
ELEMENT_MASS = {"H": 1.008, "C": 12.011, "O": 15.999}

# Constants used only to draw thermal initial momenta (CODATA 2018).
_KB_EV_PER_K = 8.617333262e-5
_AMU_A2_PER_FS2_IN_EV = 103.64269652680505

CUTOFF_A = 6.0

ZETAS = (1, 2, 4, 8)
LAMBDAS = (1.0, -1.0)


@dataclass
class Model:
    """Per-element Behler-Parrinello network and its descriptor grid.

    Feature order (D features per centre atom):
      radial block first, index e * n_rad + s for neighbour element e and
      radial function s;
      then one angular block per unordered neighbour-element pair (e1 <= e2)
      in lexicographic order, index within the block
      (i_eta * len(ZETAS) + i_zeta) * len(LAMBDAS) + i_lambda.
    Layers: W[l] has shape [out, in] (float32), b[l] shape [out]; the last
    layer has out = 1.
    angular: "g4" (angular functions with the r_jk factors) or "g5" (without
    them; same feature layout).
    """
    elements: list
    masses: np.ndarray
    cutoff: float
    rad_center: np.ndarray
    rad_eta: np.ndarray
    ang_eta: np.ndarray
    hidden: list
    weights: list           # weights[e] = [(W0, b0), (W1, b1), ..., (Wout, bout)]
    feat_shift: np.ndarray  # [n_el, D] float32
    feat_scale: np.ndarray  # [n_el, D] float32
    angular: str = "g4"

    @property
    def n_elements(self):
        return len(self.elements)

    @property
    def n_rad(self):
        return len(self.rad_center)

    @property
    def n_ang(self):
        return len(self.ang_eta) * len(ZETAS) * len(LAMBDAS)

    @property
    def n_pairs(self):
        n = self.n_elements
        return n * (n + 1) // 2

    @property
    def n_features(self):
        return self.n_elements * self.n_rad + self.n_pairs * self.n_ang


@dataclass
class System:
    n_atoms: int
    n_beads: int
    temperature: float
    box: np.ndarray          # [3]; zeros for a non-periodic system
    species: np.ndarray      # [n_atoms] int32 index into the element table
    q0: np.ndarray           # [n_atoms, 3] float64 classical geometry


@dataclass
class Workload:
    name: str
    systems: list
    model: Model
    dt: float
    tau0: float
    pile_lambda: float
    n_steps: int
    philox_seed: int
    momentum_seed: int
    extra: dict = field(default_factory=dict)

    @property
    def bead_atoms(self):
        return sum(s.n_atoms * s.n_beads for s in self.systems)


# ----------------------------------------------------------------------------
# descriptor grid and random network
# ----------------------------------------------------------------------------

def radial_grid(n_rad, r_lo=0.8, r_hi=5.5):
    """Shifted Gaussians: centres evenly spaced on [r_lo, r_hi], width = spacing."""
    spacing = (r_hi - r_lo) / (n_rad - 1)
    centres = r_lo + spacing * np.arange(n_rad, dtype=np.float64)
    etas = np.full(n_rad, 1.0 / (2.0 * spacing * spacing))
    return centres, etas


def angular_etas(n_ang):
    if n_ang == 8:
        return np.array([0.01])
    if n_ang == 16:
        return np.array([0.005, 0.02])
    raise ValueError("n_ang must be 8 or 16")


def _bfloat16_values(a):
    """float32 array rounded to the nearest bfloat16 value (ties to even), kept as float32."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def make_model(elements, n_rad, n_ang, hidden, seed, rad_scale=1.0, ang_scale=1.0, bf16_weights=True):
    """Random-weight network, W ~ N(0, 1/fan_in), zero biases.  With
    bf16_weights (the default) every weight is rounded to the nearest bfloat16
    value: the weights are still float32 numbers, the same for every precision
    and for the oracle, and a BF16 MLP then splits only its activations.

    feat_shift = 0; feat_scale is a per-block constant (radial / angular)
    chosen so the normalised features of the synthetic geometries are O(1).
    """
    rng = np.random.default_rng(seed)
    rc, re = radial_grid(n_rad)
    ae = angular_etas(n_ang)
    n_el = len(elements)
    n_pairs = n_el * (n_el + 1) // 2
    D = n_el * n_rad + n_pairs * n_ang
    weights = []
    for _e in range(n_el):
        layers = []
        fan_in = D
        for width in list(hidden) + [1]:
            W = rng.normal(0.0, 1.0 / math.sqrt(fan_in), size=(width, fan_in)).astype(np.float32)
            if bf16_weights:
                W = _bfloat16_values(W)
            b = np.zeros(width, dtype=np.float32)
            layers.append((W, b))
            fan_in = width
        weights.append(layers)
    shift = np.zeros((n_el, D), dtype=np.float32)
    scale = np.empty((n_el, D), dtype=np.float32)
    scale[:, : n_el * n_rad] = rad_scale
    scale[:, n_el * n_rad:] = ang_scale
    return Model(elements=list(elements),
                 masses=np.array([ELEMENT_MASS[e] for e in elements]),
                 cutoff=CUTOFF_A, rad_center=rc, rad_eta=re, ang_eta=ae,
                 hidden=list(hidden), weights=weights,
                 feat_shift=shift, feat_scale=scale)


@dataclass
class GfnModel:
    """Random weights of a direct-force head in the form of the paper's graph
    field network (node and edge representations exchanging messages, forces
    read out per edge).  Shapes (float32; hidden width H, L layers):
      node_embed [n_el, H], pair_embed [n_el, n_el, H] (symmetric), edge_in [H, n_rad]
      per layer: msg = (W1 [H, H], b1 [H], W2 [H, H], b2 [H]),
                 node = (W1 [H, 2H], b1, W2 [H, H], b2), edge = (W1 [H, H], b1, W2 [H, H], b2)
      force = (W1 [H, H], b1 [H], w2 [H], b2 scalar)
    The radial basis of an edge uses the grid rad_center / rad_eta."""
    elements: list
    masses: np.ndarray
    cutoff: float
    rad_center: np.ndarray
    rad_eta: np.ndarray
    width: int
    node_embed: np.ndarray
    pair_embed: np.ndarray
    edge_in: np.ndarray
    layers: list            # [(msg, node, edge)] per layer, each a (W1, b1, W2, b2) tuple
    force: tuple

    @property
    def n_elements(self):
        return len(self.elements)

    @property
    def n_rad(self):
        return len(self.rad_center)

    @property
    def n_layers(self):
        return len(self.layers)


def make_gfn_model(elements, n_rad, width, n_layers, seed):
    """Weights ~ N(0, 1/fan_in), embeddings ~ N(0, 1) (pair embeddings
    symmetrised), zero biases; the readout vector w2 ~ N(0, 0.09/H), which
    puts the rms force of the water workloads near 0.3 eV/A, the scale of the
    energy network's forces (a head without an energy is not conservative, so
    larger random forces heat the ring polymer quickly)."""
    rng = np.random.default_rng(seed)
    rc, re = radial_grid(n_rad)
    n_el, H = len(elements), width

    def lin(n_out, n_in):
        return (rng.normal(0.0, 1.0 / math.sqrt(n_in), size=(n_out, n_in)).astype(np.float32),
                np.zeros(n_out, dtype=np.float32))

    def mlp(n_in):
        W1, b1 = lin(H, n_in)
        W2, b2 = lin(H, H)
        return (W1, b1, W2, b2)

    node_embed = rng.normal(0.0, 1.0, size=(n_el, H)).astype(np.float32)
    pe = rng.normal(0.0, 1.0, size=(n_el, n_el, H))
    pair_embed = (0.5 * (pe + pe.transpose(1, 0, 2))).astype(np.float32)
    edge_in = lin(H, n_rad)[0]
    layers = [(mlp(H), mlp(2 * H), mlp(H)) for _ in range(n_layers)]
    W1, b1 = lin(H, H)
    w2 = rng.normal(0.0, 0.3 / math.sqrt(H), size=H).astype(np.float32)
    return GfnModel(elements=list(elements), masses=np.array([ELEMENT_MASS[e] for e in elements]),
                    cutoff=CUTOFF_A, rad_center=rc, rad_eta=re, width=H, node_embed=node_embed,
                    pair_embed=pair_embed, edge_in=edge_in, layers=layers,
                    force=(W1, b1, w2, np.float32(0.0)))


def gfn_workload(c, width=16, n_layers=2, seed_offset=0):
    """Workload c with the direct-force head in place of the energy network
    (same systems, seeds shifted by 500 for the head's weights)."""
    wl = workload(c, seed_offset)
    head = make_gfn_model(wl.model.elements, wl.model.n_rad, width, n_layers, 2500 + c + seed_offset)
    return Workload(wl.name + "-gfn", wl.systems, head, wl.dt, wl.tau0, wl.pile_lambda, wl.n_steps,
                    wl.philox_seed, wl.momentum_seed)


def with_g5(wl):
    """The same workload with the G5 angular functions in the descriptor
    network (no r_jk factors: every neighbour pair counts, so the angular sums
    are larger and their block scale grows, 1.5x for the formic-acid model,
    3x for water, to keep the normalised features O(1))."""
    m = wl.model
    factor = 1.5 if "C" in m.elements else 3.0
    scale = m.feat_scale.copy()
    scale[:, m.n_elements * m.n_rad:] *= np.float32(factor)
    model = dataclasses.replace(m, angular="g5", feat_scale=scale)
    return dataclasses.replace(wl, name=wl.name + "-g5", model=model)


# ----------------------------------------------------------------------------
# geometries
# ----------------------------------------------------------------------------

def formic_acid_dimer():
    """Planar cyclic formic-acid dimer with an inversion centre at the origin.

    Bond lengths: C=O 1.22, C-O 1.31, O-H 0.98, C-H 1.09 A;
    the two O-H...O hydrogen bonds have O...O = 2.70 A.
    Returns (elements, species, positions) with the element table [H, C, O];
    atom order per monomer: C, O(carbonyl), O(hydroxyl), H(formyl), H(hydroxyl).
    """
    def monomer(half_sep):
        C = np.array([-half_sep, 0.0, 0.0])
        Oc = C + 1.22 * np.array([math.cos(math.radians(60)), math.sin(math.radians(60)), 0.0])
        Oh = C + 1.31 * np.array([math.cos(math.radians(-60)), math.sin(math.radians(-60)), 0.0])
        Hf = C + 1.09 * np.array([-1.0, 0.0, 0.0])
        return C, Oc, Oh, Hf

    # solve for the C...C half separation giving O(c, A)...O(h, B) = 2.70 A
    lo, hi = 1.0, 4.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        _, Oc, Oh, _ = monomer(mid)
        OhB = -Oh
        if np.linalg.norm(OhB - Oc) < 2.70:
            lo = mid
        else:
            hi = mid
    C, Oc, Oh, Hf = monomer(0.5 * (lo + hi))
    CB, OcB, OhB, HfB = -C, -Oc, -Oh, -Hf
    Hh = Oh + 0.98 * (OcB - Oh) / np.linalg.norm(OcB - Oh)     # A's hydroxyl H points at B's C=O
    HhB = -Hh
    pos = np.array([C, Oc, Oh, Hf, Hh, CB, OcB, OhB, HfB, HhB])
    elements = ["H", "C", "O"]
    species = np.array([1, 2, 2, 0, 0, 1, 2, 2, 0, 0], dtype=np.int32)
    return elements, species, pos


def _random_rotation(rng):
    u1, u2, u3 = rng.random(3)
    a = math.sqrt(1 - u1)
    b = math.sqrt(u1)
    x, y, z, w = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2), \
        b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _water_body(r_oh=0.96, angle_deg=104.52):
    h = math.radians(angle_deg) / 2
    return np.array([[0.0, 0.0, 0.0],
                     [r_oh * math.sin(h), r_oh * math.cos(h), 0.0],
                     [-r_oh * math.sin(h), r_oh * math.cos(h), 0.0]])


def _min_image(d, box):
    return d - box * np.round(d / box)


def water_grid(n_side, box_len, rng, min_sep=1.0):
    """n_side^3 water molecules, O on a simple cubic grid, random orientations.

    An orientation is redrawn while any intermolecular atom pair (minimum
    image) is closer than min_sep.  Element table [H, O]; order O, H, H.
    """
    box = np.full(3, box_len)
    spacing = box_len / n_side
    body = _water_body()
    placed = np.zeros((0, 3))
    pos = []
    for ix in range(n_side):
        for iy in range(n_side):
            for iz in range(n_side):
                o = spacing * (np.array([ix, iy, iz]) + 0.5)
                for _attempt in range(1000):
                    mol = o + body @ _random_rotation(rng).T
                    if len(placed) == 0:
                        break
                    d = _min_image(mol[:, None, :] - placed[None, :, :], box)
                    if np.min(np.einsum("ijk,ijk->ij", d, d)) >= min_sep * min_sep:
                        break
                else:
                    raise RuntimeError("could not place water molecule")
                pos.append(mol)
                placed = np.concatenate([placed, mol])
    pos = np.concatenate(pos)
    species = np.tile(np.array([1, 0, 0], dtype=np.int32), n_side ** 3)
    return ["H", "O"], species, pos, box


ICE_FRACTIONAL = np.array([
    [0.0, 1 / 3, 1 / 16], [0.0, 1 / 3, 7 / 16],
    [0.5, 1 / 6, 9 / 16], [0.5, 1 / 6, 15 / 16],
    [0.5, 5 / 6, 1 / 16], [0.5, 5 / 6, 7 / 16],
    [0.0, 2 / 3, 9 / 16], [0.0, 2 / 3, 15 / 16]])


def ice_oxygens(a=4.5, c=7.35, reps=(3, 2, 2)):
    """O sublattice of hexagonal ice in an orthorhombic (a, a*sqrt3, c) cell."""
    cell = np.array([a, a * math.sqrt(3.0), c])
    pts = []
    for i in range(reps[0]):
        for j in range(reps[1]):
            for k in range(reps[2]):
                pts.append((ICE_FRACTIONAL + np.array([i, j, k])) * cell)
    return np.concatenate(pts), cell * np.array(reps)


def ice_ih(rng, r_oh=0.96, bond_cut=3.0, n_flips_per_o=10):
    """Proton-disordered ice-Ih obeying the ice rules.

    The O-O hydrogen-bond graph is 4-regular.  Orienting every edge along a
    seeded random Euler circuit gives each O two donated and two accepted
    bonds; random directed-loop reversals then decorrelate the arrangement.
    Each donated bond carries one H at r_oh from the donor.
    Element table [H, O]; atom order per molecule O, H, H.
    """
    O, box = ice_oxygens()
    n = len(O)
    d = _min_image(O[:, None, :] - O[None, :, :], box)
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    nbrs = [list(np.nonzero((r[i] < bond_cut) & (np.arange(n) != i))[0]) for i in range(n)]
    if any(len(v) != 4 for v in nbrs):
        raise RuntimeError("ice O graph is not 4-regular")
    # Hierholzer's algorithm with random edge choice
    unused = {i: list(v) for i, v in enumerate(nbrs)}
    for v in unused.values():
        rng.shuffle(v)
    stack, circuit = [0], []
    while stack:
        v = stack[-1]
        if unused[v]:
            w = unused[v].pop()
            unused[w].remove(v)
            stack.append(w)
        else:
            circuit.append(stack.pop())
    succ = {i: set() for i in range(n)}
    for a, b in zip(circuit[:-1], circuit[1:]):
        succ[b].add(a)   # circuit was built in reverse; orientation b -> a
    # directed-loop reversals keep in = out = 2 everywhere
    for _ in range(n_flips_per_o * n):
        start = int(rng.integers(n))
        path, seen = [start], {start: 0}
        while True:
            nxt = list(succ[path[-1]])
            w = nxt[int(rng.integers(len(nxt)))]
            if w in seen:
                loop = path[seen[w]:] + [w]
                break
            seen[w] = len(path)
            path.append(w)
        for a, b in zip(loop[:-1], loop[1:]):
            succ[a].remove(b)
            succ[b].add(a)
    pos = []
    for i in range(n):
        donors = sorted(succ[i])
        assert len(donors) == 2
        mol = [O[i]]
        for j in donors:
            v = _min_image(O[j] - O[i], box)
            mol.append(O[i] + r_oh * v / np.linalg.norm(v))
        pos.append(np.array(mol))
    species = np.tile(np.array([1, 0, 0], dtype=np.int32), n)
    return ["H", "O"], species, np.concatenate(pos), box


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def _fad_system(rng, n_beads, temperature):
    elements, species, pos = formic_acid_dimer()
    q0 = pos + rng.uniform(-0.05, 0.05, size=pos.shape)
    return elements, System(n_atoms=len(species), n_beads=n_beads, temperature=temperature,
                            box=np.zeros(3), species=species, q0=q0)


# Feature scales: angular blocks are sums over O(K^2) triplets, so they are
# divided by a per-workload constant that brings them to O(1).
_FAD_SCALES = dict(rad_scale=1.0, ang_scale=1.0)
_WATER_SCALES = dict(rad_scale=2.0, ang_scale=10.0)


def workload(c, seed_offset=0, bf16_weights=True):
    """Build workload number c (1..5) as described in the module docstring.

    Seeds: geometry 1000+c, weights 2000+c, momenta 3000+c, Philox 4000+c,
    each shifted by seed_offset (parity tests use 0, 100, 200).
    bf16_weights: see make_model.
    """
    gs, ws, ms, ps = (1000 + c + seed_offset, 2000 + c + seed_offset,
                      3000 + c + seed_offset, 4000 + c + seed_offset)
    rng = np.random.default_rng(gs)
    if c == 1:
        elements, sys1 = _fad_system(rng, 8, 300.0)
        model = make_model(elements, 8, 8, [64, 64], ws, bf16_weights=bf16_weights, **_FAD_SCALES)
        return Workload("fad-10atom-P8", [sys1], model, dt=0.25, tau0=100.0, pile_lambda=1.0,
                        n_steps=500, philox_seed=ps, momentum_seed=ms)
    if c == 2:
        elements, species, pos, box = water_grid(4, 12.42, rng)
        s = System(len(species), 32, 300.0, box, species, pos)
        model = make_model(elements, 16, 16, [128, 128, 64], ws, bf16_weights=bf16_weights, **_WATER_SCALES)
        return Workload("water-64-P32", [s], model, dt=0.25, tau0=100.0, pile_lambda=1.0,
                        n_steps=200, philox_seed=ps, momentum_seed=ms)
    if c == 3:
        elements, species, pos, box = ice_ih(rng)
        s = System(len(species), 32, 250.0, box, species, pos)
        model = make_model(elements, 16, 16, [128, 128, 64], ws, bf16_weights=bf16_weights, **_WATER_SCALES)
        return Workload("ice-96-P32", [s], model, dt=0.25, tau0=100.0, pile_lambda=1.0,
                        n_steps=4000, philox_seed=ps, momentum_seed=ms)
    if c == 4:
        systems = []
        elements = None
        for _ in range(512):
            p = int(rng.choice([8, 16, 32, 64]))
            t = float(rng.uniform(100.0, 400.0))
            elements, s = _fad_system(rng, p, t)
            systems.append(s)
        model = make_model(elements, 8, 8, [64, 64], ws, bf16_weights=bf16_weights, **_FAD_SCALES)
        return Workload("fad-batch-512", systems, model, dt=0.25, tau0=100.0, pile_lambda=1.0,
                        n_steps=200, philox_seed=ps, momentum_seed=ms)
    if c == 5:
        elements, species, pos, box = water_grid(16, 49.7, rng)
        s = System(len(species), 32, 300.0, box, species, pos)
        model = make_model(elements, 16, 16, [128, 128, 64], ws, bf16_weights=bf16_weights, **_WATER_SCALES)
        return Workload("water-4096-P32", [s], model, dt=0.25, tau0=100.0, pile_lambda=1.0,
                        n_steps=200, philox_seed=ps, momentum_seed=ms)
    raise ValueError(f"unknown workload {c}")


def small_workload(kind, seed=7, n_beads=4, bf16_weights=True):
    """Small variants for fast tests: 'fad' (10 atoms), 'water8' (8 H2O in a
    periodic 12.5 A box, so the cell grid is 2x2x2 and stencils wrap)."""
    rng = np.random.default_rng(seed)
    if kind == "fad":
        elements, s = _fad_system(rng, n_beads, 300.0)
        model = make_model(elements, 8, 8, [64, 64], seed + 1, bf16_weights=bf16_weights, **_FAD_SCALES)
        return Workload("fad-small", [s], model, 0.25, 100.0, 1.0, 10, seed + 2, seed + 3)
    if kind == "water8":
        elements, species, pos, box = water_grid(2, 12.5, rng)
        s = System(len(species), n_beads, 300.0, box, species, pos)
        model = make_model(elements, 16, 16, [128, 128, 64], seed + 1, bf16_weights=bf16_weights, **_WATER_SCALES)
        return Workload("water8", [s], model, 0.25, 100.0, 1.0, 10, seed + 2, seed + 3)
    raise ValueError(kind)


def colliding_clusters(n_beads=4, speed=0.08, seed=7, box_len=24.0):
    """Two clusters of three water molecules flying at each other along x in a
    periodic box (a neighbour count that grows during a run, for the overflow
    tests).  O atoms on an equilateral triangle of side 2.9 A in the yz plane
    with random molecule orientations; cluster centres 12 A apart, so every
    atom starts with the 8 other atoms of its cluster as its only neighbours
    within 6 A.  Returns (workload, q, p): every bead at the geometry, momenta
    m v along +x (first cluster) and -x (second), no thermal part; NVE,
    dt = 0.5 fs, the water model of small_workload("water8")."""
    rng = np.random.default_rng(seed)
    body = _water_body()
    tri = 2.9 / math.sqrt(3.0) * np.array([[0.0, math.cos(a), math.sin(a)]
                                           for a in (0.0, 2 * math.pi / 3, 4 * math.pi / 3)])
    centre = np.array([box_len / 2, box_len / 2, box_len / 2])
    pos, vel = [], []
    for dx, v in ((-6.0, speed), (6.0, -speed)):
        for o in tri:
            pos.append(centre + np.array([dx, 0.0, 0.0]) + o + body @ _random_rotation(rng).T)
            vel.append(np.full(3, v))
    pos = np.concatenate(pos)
    species = np.tile(np.array([1, 0, 0], dtype=np.int32), 6)
    box = np.full(3, box_len)
    model = small_workload("water8").model
    s = System(len(species), n_beads, 300.0, box, species, pos)
    wl = Workload("colliding-clusters", [s], model, 0.5, 0.0, 1.0, 200, seed + 2, seed + 3)
    m = model.masses[species]
    vx = np.concatenate([np.full(9, speed), np.full(9, -speed)])
    p1 = np.zeros((len(species), 3))
    p1[:, 0] = m * vx
    q = np.broadcast_to(pos, (n_beads, len(species), 3)).reshape(-1, 3)
    p = np.broadcast_to(p1, (n_beads, len(species), 3)).reshape(-1, 3)
    return wl, q.astype(np.float32), p.astype(np.float32)


def initial_state(wl):
    """All beads at the classical geometry (unwrapped) and thermal bead momenta
    p ~ N(0, m kB T P), drawn with numpy default_rng(momentum_seed).

    Returns q, p as float32 arrays [sum_s P_s N_s, 3] in the bead-major,
    system-concatenated layout (index off_s + k * N_s + i).
    """
    rng = np.random.default_rng(wl.momentum_seed)
    qs, ps = [], []
    masses = wl.model.masses
    for s in wl.systems:
        m = masses[s.species]
        q = np.broadcast_to(s.q0, (s.n_beads, s.n_atoms, 3))
        sd = np.sqrt(m * _KB_EV_PER_K * s.temperature * s.n_beads / _AMU_A2_PER_FS2_IN_EV)
        p = rng.normal(size=(s.n_beads, s.n_atoms, 3)) * sd[None, :, None]
        qs.append(q.reshape(-1, 3))
        ps.append(p.reshape(-1, 3))
    return (np.concatenate(qs).astype(np.float32), np.concatenate(ps).astype(np.float32))


def perturbed_beads(wl, amplitude=0.05, seed=11):
    """Bead positions with independent jitter per bead (so the beads differ),
    float32 [sum P_s N_s, 3]; used for force-parity tests."""
    rng = np.random.default_rng(seed)
    qs = []
    for s in wl.systems:
        q = s.q0[None] + rng.uniform(-amplitude, amplitude, size=(s.n_beads, s.n_atoms, 3))
        qs.append(q.reshape(-1, 3))
    return np.concatenate(qs).astype(np.float32)


# ----------------------------------------------------------------------------
# well-tempered metadynamics settings (Sec. 2.5; S2 and S3 sampling paragraphs)
# ----------------------------------------------------------------------------

# 1 eV = 96.48533212 kJ/mol (CODATA 2018 Faraday constant).
KJ_PER_MOL_IN_EV = 1.0 / 96.48533212

# X-ray atomic scattering factors as four-Gaussian fits,
# f(s) = sum_i a_i exp(-b_i s^2) + c with s = sin(theta)/lambda = Q/(4 pi)
# (Cromer-Mann coefficients as tabulated in International Tables for
# Crystallography Vol. C, Table 6.1.1.4); only f at one Q enters a run.
_CROMER_MANN = {
    "H": ((0.489918, 0.262003, 0.196767, 0.049879), (20.6593, 7.74039, 49.5519, 2.20159), 0.001305),
    "C": ((2.31, 1.02, 1.5886, 0.865), (20.8439, 10.2075, 0.5687, 51.6512), 0.2156),
    "O": ((3.0485, 2.2868, 1.5463, 0.867), (13.2771, 5.7011, 0.3239, 32.9089), 0.2508),
}


def scattering_factor(element, Q):
    """X-ray form factor of an element at scattering vector Q (1/A)."""
    a, b, c = _CROMER_MANN[element]
    s2 = (Q / (4.0 * math.pi)) ** 2
    return float(sum(ai * math.exp(-bi * s2) for ai, bi in zip(a, b)) + c)


def scattering_vector(theta_deg, wavelength_A):
    """Q = 4 pi sin(theta) / lambda (1/A)."""
    return 4.0 * math.pi * math.sin(math.radians(theta_deg)) / wavelength_A


# Double proton transfer in the dimer (Sec. 3.1): with the atom order of
# formic_acid_dimer(), H(1) = 4 is bound to O(1) = 2 (monomer A hydroxyl) and
# points at O(2) = 6 (monomer B carbonyl); H(2) = 9 is bound to O(4) = 7 and
# points at O(3) = 1.  s = d(O1,H1) - d(O2,H1) + d(O4,H2) - d(O3,H2) is
# -1.48 A in the reactant geometry and +1.48 A after both protons moved.
FAD_DPT_ATOMS = np.array([[2, 4], [6, 4], [7, 9], [1, 9]], dtype=np.int32)
FAD_DPT_COEF = np.array([1.0, -1.0, 1.0, -1.0])


@dataclass
class MetadSpec:
    """Collective variable and well-tempered deposition settings.

    cv "distances": s = sum_m coef[m] |r_atoms[m,0] - r_atoms[m,1]| (A);
    cv "xrd": S = (1/N) sum_ij f_i f_j sinc(Q R_ij) with form_factor[element].
    height0 in eV, sigma in CV units, stride in steps, max_hills per bead."""
    cv: str
    atoms: np.ndarray = None
    coef: np.ndarray = None
    q_scatter: float = 0.0
    form_factor: np.ndarray = None
    height0: float = 1.0 * KJ_PER_MOL_IN_EV
    sigma: float = 0.05
    gamma: float = 10.0
    stride: int = 100
    max_hills: int = 1024


def metad_spec(wl, stride=None, max_hills=1024):
    """The sampling settings of the paper's two studies for a workload:
    dimer systems use s_dimer (S2: hill every 100 steps, 1 kJ/mol, bias
    factor 10); water and ice use the XRD CV at theta = 11.95 deg,
    lambda = 1.54 A (S3: hill every 0.05 ps, 1 kJ/mol, bias factor 60).
    The widths are not given in the paper: 0.05 A for s_dimer and 0.05
    (electrons^2) for S, small against each CV's spread over the beads of a
    thermal ring polymer."""
    if "C" in wl.model.elements:
        return MetadSpec("distances", atoms=FAD_DPT_ATOMS.copy(), coef=FAD_DPT_COEF.copy(), sigma=0.05,
                         gamma=10.0, stride=stride or 100, max_hills=max_hills)
    Q = scattering_vector(11.95, 1.54)
    f = np.array([scattering_factor(e, Q) for e in wl.model.elements])
    return MetadSpec("xrd", q_scatter=Q, form_factor=f, sigma=0.05, gamma=60.0,
                     stride=stride or int(round(50.0 / wl.dt)), max_hills=max_hills)
