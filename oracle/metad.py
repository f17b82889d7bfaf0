"""Well-tempered metadynamics on bead collective variables (FP64, oracle
side; test infrastructure only).

Sec. 2.5 adds to the Hamiltonian a bias V_G(s, t) built from Gaussian kernels
laid along the trajectory of a collective variable s(R), the height of each
kernel shrinking with the bias already present at its centre (well-tempered
form, bias factor gamma), so that the bias converges to -(1 - 1/gamma) F(s).
For the quantum system the free-energy surface is a reweighting over the P
beads: F_q(s) = -1/beta ln[(1/P) sum_k exp(-beta F^(k)(s))].

Readings written out here (each is listed in the design notes):

  * Each bead k of a ring polymer carries its own bias V^(k), built from the
    hills deposited at its own CV values s^(k) = s(r^(k)); F^(k) in the
    reweighting is the free energy that bias estimates,
    F^(k)(s) = -(gamma / (gamma - 1)) V^(k)(s).
  * The bias of bead k enters that bead's potential the way the physical
    potential does: bead potential V(r^(k)) + V^(k)(s(r^(k))), so with all
    beads at one point the ring feels the bead-averaged bias at the physical
    beta, and P = 1 is classical WT-MetaD.
  * Deposition is discrete: after every `stride` completed steps each bead
    adds a hill at its current CV value, of height
        h = w0 exp(-beta V^(k)(s^(k)) / (gamma - 1)),
    beta = 1 / (k_B T) of the system, V^(k) the bias before the new hill.
    The forces of the step that deposits use the bias before the hill.
  * Kernel: exp(-(s - c)^2 / (2 sigma^2)) with sigma the width in CV units
    (the paper prints 2 sigma in the denominator; sigma^2 is read).
  * CVs (Sec. 3.1, Sec. 3.2 and the S2, S3 sampling paragraphs):
      distances:  s = sum_m c_m |r_a(m) - r_b(m)|   (s_dimer: c = +1, -1, +1, -1)
      XRD:        S = (1/N) sum_i sum_j f_i f_j sinc(Q R_ij),  sinc(x) = sin(x)/x, sinc(0) = 1,
                  over all ordered pairs including i = j, Q = 4 pi sin(theta) / lambda.
    In a periodic box every distance is the minimum-image distance (the
    paper states R_ij = |R_i - R_j| and no cutoff or window).
"""
import numpy as np

from .constants import KB


def _displacements(q, box, a, b):
    """r_a - r_b (minimum image when the box is periodic), FP64."""
    d = np.asarray(q, dtype=np.float64)[a] - np.asarray(q, dtype=np.float64)[b]
    box = np.asarray(box, dtype=np.float64)
    if np.any(box > 0):
        d = d - box * np.round(d / box)
    return d


def cv_distances(q, box, atoms, coef):
    """s = sum_m coef[m] |r_atoms[m,0] - r_atoms[m,1]| of one bead and ds/dr [N, 3]."""
    q = np.asarray(q, dtype=np.float64)
    atoms = np.asarray(atoms, dtype=np.int64).reshape(-1, 2)
    coef = np.asarray(coef, dtype=np.float64)
    d = _displacements(q, box, atoms[:, 0], atoms[:, 1])
    r = np.sqrt(np.sum(d * d, axis=1))
    s = float(np.sum(coef * r))
    grad = np.zeros_like(q)
    u = coef[:, None] * d / r[:, None]
    np.add.at(grad, atoms[:, 0], u)
    np.add.at(grad, atoms[:, 1], -u)
    return s, grad


def sinc(x):
    """sin(x)/x with the limit 1 at x = 0."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = x != 0
    out[nz] = np.sin(x[nz]) / x[nz]
    return out


def dsinc(x):
    """d sinc / dx = (x cos x - sin x) / x^2, 0 at x = 0."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    xn = x[nz]
    out[nz] = (xn * np.cos(xn) - np.sin(xn)) / (xn * xn)
    return out


def xrd_row(q, species, box, Q, f, i):
    """Row i of the double sum, sum_j f_i f_j sinc(Q R_ij), and dS/dr_i [3]
    (both orderings of every pair involving i)."""
    q = np.asarray(q, dtype=np.float64)
    fa = np.asarray(f, dtype=np.float64)[np.asarray(species)]
    n = len(q)
    d = _displacements(q, box, np.full(n, i), np.arange(n))     # r_i - r_j
    R = np.sqrt(np.sum(d * d, axis=1))
    row = fa[i] * np.sum(fa * sinc(Q * R))
    w = np.zeros(n)
    nz = R > 0
    w[nz] = fa[i] * fa[nz] * Q * dsinc(Q * R[nz]) / R[nz]
    grad = 2.0 * np.sum(w[:, None] * d, axis=0) / n
    return row, grad


def cv_xrd(q, species, box, Q, f, rows=None):
    """S of one bead and dS/dr [N, 3] (rows None: every atom; else only the
    listed atoms' gradients are filled, S is always the full sum)."""
    q = np.asarray(q, dtype=np.float64)
    n = len(q)
    S = 0.0
    grad = np.zeros_like(q)
    want = set(range(n)) if rows is None else set(int(r) for r in rows)
    for i in range(n):
        row, g = xrd_row(q, species, box, Q, f, i)
        S += row
        if i in want:
            grad[i] = g
    return S / n, grad


def bias(s, centers, heights, sigma):
    """V(s) = sum_h heights[h] exp(-(s - centers[h])^2 / (2 sigma^2)) and dV/ds."""
    c = np.asarray(centers, dtype=np.float64)
    h = np.asarray(heights, dtype=np.float64)
    if len(c) == 0:
        return 0.0, 0.0
    x = (s - c) / sigma
    g = h * np.exp(-0.5 * x * x)
    return float(np.sum(g)), float(np.sum(-g * x / sigma))


def well_tempered_height(v_here, temperature, w0, gamma):
    """Height of a new hill where the bias is already v_here."""
    if np.isinf(gamma):
        return float(w0)
    return float(w0 * np.exp(-v_here / (KB * temperature * (gamma - 1.0))))


def fes_quantum(grid, centers, heights, sigma, gamma, temperature):
    """F_q(s) on a grid from the P bead biases (centers, heights: [P][n]),
    F^(k) = -(gamma / (gamma - 1)) V^(k), reweighted over the beads."""
    beta = 1.0 / (KB * temperature)
    P = len(centers)
    Fk = np.array([[-(gamma / (gamma - 1.0)) * bias(s, centers[k], heights[k], sigma)[0] for s in grid]
                   for k in range(P)])
    m = np.min(Fk, axis=0)
    return m - np.log(np.mean(np.exp(-beta * (Fk - m[None, :])), axis=0)) / beta


class Metad:
    """Per-bead hill histories of a list of ring polymers and the biased
    force function handed to the ring-polymer integrator.

    systems: list of (n_atoms, n_beads, temperature, species, box).
    cv: ("distances", atoms [M, 2], coef [M]) or ("xrd", Q, f[n_elements]).
    The state layout matches the integrator: index off_s + k N_s + i.
    """

    def __init__(self, systems, cv, w0, sigma, gamma, stride):
        self.systems = systems
        self.cv = cv
        self.w0, self.sigma, self.gamma, self.stride = w0, sigma, gamma, stride
        self.offsets = np.cumsum([0] + [n * P for n, P, _, _, _ in systems])
        self.n_beads = sum(P for _, P, _, _, _ in systems)
        self.centers = [[] for _ in range(self.n_beads)]
        self.heights = [[] for _ in range(self.n_beads)]
        self.last_s = np.zeros(self.n_beads)
        self.last_v = np.zeros(self.n_beads)

    def beads(self):
        """(global bead, system, first row, atoms) of every bead."""
        g = 0
        for si, (n, P, _, _, _) in enumerate(self.systems):
            for k in range(P):
                yield g, si, int(self.offsets[si]) + k * n, n
                g += 1

    def bead_cv(self, q, si, row0, n, rows=None):
        _, _, _, species, box = self.systems[si]
        qb = np.asarray(q, dtype=np.float64)[row0:row0 + n]
        if self.cv[0] == "distances":
            return cv_distances(qb, box, self.cv[1], self.cv[2])
        return cv_xrd(qb, species, box, self.cv[1], self.cv[2], rows)

    def bias_forces(self, q):
        """CV and bias energy per bead and the bias forces [rows, 3] at q."""
        q = np.asarray(q, dtype=np.float64)
        F = np.zeros_like(q)
        s_all, v_all = np.zeros(self.n_beads), np.zeros(self.n_beads)
        for g, si, row0, n in self.beads():
            s, grad = self.bead_cv(q, si, row0, n)
            v, dv = bias(s, self.centers[g], self.heights[g], self.sigma)
            F[row0:row0 + n] = -dv * grad
            s_all[g], v_all[g] = s, v
        return s_all, v_all, F

    def force_fn(self, base_fn):
        """Physical forces plus the bias forces of the current hills."""
        def fn(q):
            E, F = base_fn(q)
            s, v, Fb = self.bias_forces(q)
            self.last_s, self.last_v = s, v
            return E, F + Fb
        return fn

    def deposit(self):
        """One hill per bead at the CV of the last force evaluation."""
        for g, si, _, _ in self.beads():
            T = self.systems[si][2]
            self.centers[g].append(float(self.last_s[g]))
            self.heights[g].append(well_tempered_height(self.last_v[g], T, self.w0, self.gamma))

    def step(self, rp, noise=None):
        """One integrator step of rp (built with force_fn) and the deposition
        that follows it when the completed step count is a multiple of stride."""
        rp.step(noise=noise)
        if rp.step_count % self.stride == 0:
            self.deposit()

    def fes(self, si, grid):
        """Quantum free-energy surface of system si on a grid."""
        b0 = sum(P for _, P, _, _, _ in self.systems[:si])
        P = self.systems[si][1]
        return fes_quantum(grid, self.centers[b0:b0 + P], self.heights[b0:b0 + P], self.sigma, self.gamma,
                           self.systems[si][2])
