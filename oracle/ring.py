"""Ring-polymer dynamics in FP64 (oracle side).

Ring polymer (Sec. 2.1): P beads per atom joined by harmonic springs.  The
oracle samples exp(-beta_P H_P) with beta_P = beta / P and
  H_P = sum_k sum_i [ |p_i^k|^2 / (2 m_i) + 1/2 m_i w_P^2 |q_i^k - q_i^{k+1}|^2 ] + sum_k V(q^k),
  w_P = P k_B T / hbar  (bead index k+1 taken modulo P),
which has the same configurational distribution as the effective Hamiltonian
of Sec. 2.1 (springs with sqrt(P)/(beta hbar) and V/P at inverse temperature
beta) once the momenta are integrated out.  Physical masses are used for
every mode.

Normal modes (Sec. 2.1 and 2.3 name the normal-mode transformation): the
orthonormal matrix C with columns
  k = 0:              1/sqrt(P)
  1 <= k < P/2:       sqrt(2/P) cos(2 pi j k / P)
  k = P/2:            (-1)^j / sqrt(P)
  P/2 < k < P:        sqrt(2/P) sin(2 pi j k / P)
gives q~_k = sum_j C_jk q_j, and the free ring polymer decouples into
oscillators of frequency w_k = 2 w_P sin(k pi / P).

Integrator: PILE-L (Ceriotti, Parrinello, Markland, Manolopoulos, J. Chem.
Phys. 133, 124104 (2010)), named by Table S3, in the symmetric splitting
O(dt/2) B(dt/2) A(dt) [forces] B(dt/2) O(dt/2):
  O: p~_k <- c1_k p~_k + sqrt(m k_B T P) c2_k xi,  c1 = exp(-gamma_k dt/2), c2 = sqrt(1 - c1^2),
     gamma_0 = 1/tau0, gamma_k = 2 lambda w_k;  tau0 <= 0 switches the thermostat off;
  B: p <- p + dt/2 F;
  A: centroid drifts, every other mode rotates exactly in its phase space.
Units: A, fs, amu, eV; momenta in amu A/fs, so a kick is dt/2 F / MVV2E and
energies carry a factor MVV2E.
"""
import numpy as np

from .constants import KB, HBAR, MVV2E
from . import philox


def nm_matrix(P):
    """C[j, k] as defined in the module docstring (P = 1 or even)."""
    if P == 1:
        return np.ones((1, 1))
    if P % 2:
        raise ValueError("odd P > 1 is not supported")
    j = np.arange(P)[:, None]
    C = np.empty((P, P))
    C[:, 0] = 1.0 / np.sqrt(P)
    for k in range(1, P):
        if k < P // 2:
            C[:, k] = np.sqrt(2.0 / P) * np.cos(2 * np.pi * j[:, 0] * k / P)
        elif k == P // 2:
            C[:, k] = (-1.0) ** j[:, 0] / np.sqrt(P)
        else:
            C[:, k] = np.sqrt(2.0 / P) * np.sin(2 * np.pi * j[:, 0] * k / P)
    return C


def mode_frequencies(P, T):
    wP = P * KB * T / HBAR
    return 2.0 * wP * np.sin(np.arange(P) * np.pi / P), wP


class RingPolymers:
    """State and OBABO stepping of a list of independent ring polymers.

    systems: list of (n_atoms, n_beads, temperature, masses[n_atoms]).
    force_fn(q[sum P_s N_s, 3]) -> (E_bead[sum P_s], F[sum P_s N_s, 3]).
    State arrays use the bead-major, system-concatenated layout
    index = off_s + k N_s + i; the thermostat noise of (system, mode k, atom i)
    uses the same index as its Philox counter.
    """

    def __init__(self, systems, dt, tau0, pile_lambda, seed, force_fn, thermostat="pile-l", boxes=None):
        self.systems = systems
        self.dt, self.tau0, self.lam, self.seed = dt, tau0, pile_lambda, seed
        self.force_fn = force_fn
        if thermostat not in ("pile-l", "pile-g"):
            raise ValueError(thermostat)
        self.thermostat = thermostat
        self.boxes = None if boxes is None else np.asarray(boxes, dtype=np.float64).reshape(len(systems), 3)
        self.offsets = np.cumsum([0] + [n * P for n, P, _, _ in systems])
        self.total = int(self.offsets[-1])
        self.heat = np.zeros(len(systems))
        self.step_count = 0
        self.q = self.p = self.F = self.E = self.W = None

    def _forces(self):
        """force_fn(q) -> (E, F) or (E, F, W) with W[sum P_s, 3, 3] the bead virials."""
        out = self.force_fn(self.q)
        self.E, self.F = out[0], out[1]
        self.W = out[2] if len(out) > 2 else None

    # -- per-system views ---------------------------------------------------
    def _view(self, a, s):
        n, P, _, _ = self.systems[s]
        return a[self.offsets[s]:self.offsets[s + 1]].reshape(P, n, 3)

    def set_state(self, q, p, step=0):
        self.q = np.array(q, dtype=np.float64).reshape(-1, 3)
        self.p = np.array(p, dtype=np.float64).reshape(-1, 3)
        self.step_count = step
        self._forces()

    # -- the four sub-steps ---------------------------------------------------
    def _o_step(self, s, pt, xi):
        n, P, T, m = self.systems[s]
        wk, _ = mode_frequencies(P, T)
        glob = self.thermostat == "pile-g" and self.tau0 > 0
        if self.tau0 > 0:
            gamma = 2.0 * self.lam * wk
            gamma[0] = 0.0 if glob else 1.0 / self.tau0
        else:
            gamma = np.zeros(P)
        c1 = np.exp(-gamma * self.dt / 2)
        c2 = np.sqrt(1.0 - c1 * c1)
        sigma = np.sqrt(m * KB * T * P / MVV2E)
        ke0 = 0.5 * MVV2E * np.sum(pt * pt / m[None, :, None])
        alpha = self._svr_factor(s, pt[0], xi[0]) if glob else 1.0
        pt = c1[:, None, None] * pt + sigma[None, :, None] * c2[:, None, None] * xi
        pt[0] = alpha * pt[0]
        ke1 = 0.5 * MVV2E * np.sum(pt * pt / m[None, :, None])
        self.heat[s] -= ke1 - ke0
        return pt

    def _svr_factor(self, s, p0, xi0):
        """PILE-G: one factor for all centroid momenta of system s over a half
        step, the stochastic velocity rescaling of Bussi, Donadio and
        Parrinello (J. Chem. Phys. 126, 014101 (2007), Appendix): with
        N_f = 3N centroid degrees of freedom, centroid kinetic energy K, target
        Kbar = N_f k_B T P / 2 (the centroid momenta of the bead-potential form
        have variance m k_B T P) and c = exp(-(dt/2)/tau0),
          alpha^2 = c + (Kbar/(N_f K)) (1 - c) (R_1^2 + S) + 2 R_1 sqrt(c (1 - c) Kbar/(N_f K)),
          sign(alpha) = sign(R_1 + sqrt(c N_f K / ((1 - c) Kbar))),
        R_1 a standard normal and S a chi-square variate with N_f - 1 degrees.
        Its random numbers are the centroid's own normals of this half step:
        R_1 that of (atom 0, x), S the sum of squares of the other 3N - 1."""
        n, P, T, m = self.systems[s]
        nf = 3 * n
        K = 0.5 * MVV2E * np.sum(p0 * p0 / m[:, None])
        if K <= 0.0:
            return 1.0
        kbar = 0.5 * nf * KB * T * P
        c = np.exp(-0.5 * self.dt / self.tau0)
        r1 = float(xi0[0, 0])
        rest = float(np.sum(xi0 * xi0)) - r1 * r1
        ratio = kbar / (nf * K)
        a2 = c + ratio * (1.0 - c) * (r1 * r1 + rest) + 2.0 * r1 * np.sqrt(c * (1.0 - c) * ratio)
        sign = 1.0 if r1 + np.sqrt(c / ((1.0 - c) * ratio)) >= 0.0 else -1.0
        return sign * np.sqrt(a2)

    def _a_step(self, s, qt, pt):
        n, P, T, m = self.systems[s]
        wk, _ = mode_frequencies(P, T)
        dt = self.dt
        qn, pn = qt.copy(), pt.copy()
        qn[0] = qt[0] + dt * pt[0] / m[:, None]
        for k in range(1, P):
            c, sn = np.cos(wk[k] * dt), np.sin(wk[k] * dt)
            pn[k] = c * pt[k] - (m[:, None] * wk[k] * sn) * qt[k]
            qn[k] = sn * pt[k] / (m[:, None] * wk[k]) + c * qt[k]
        return qn, pn

    def _noise(self, half, noise):
        if noise is not None:
            return np.asarray(noise[half], dtype=np.float64).reshape(-1, 3)
        return philox.thermostat_noise(self.seed, self.step_count, half, self.total)

    def step(self, noise=None):
        """One OBABO step; noise optionally [2, total, 3] replaces Philox."""
        xi0 = self._noise(0, noise)
        for s in range(len(self.systems)):
            n, P, T, m = self.systems[s]
            C = nm_matrix(P)
            p, q, F = self._view(self.p, s), self._view(self.q, s), self._view(self.F, s)
            pt = np.einsum("jk,jnc->knc", C, p)
            pt = self._o_step(s, pt, self._view(xi0, s))
            pt = pt + (self.dt / 2) * np.einsum("jk,jnc->knc", C, F) / MVV2E
            qt = np.einsum("jk,jnc->knc", C, q)
            qt, pt = self._a_step(s, qt, pt)
            q[...] = np.einsum("jk,knc->jnc", C, qt)
            p[...] = np.einsum("jk,knc->jnc", C, pt)
        self._forces()
        xi1 = self._noise(1, noise)
        for s in range(len(self.systems)):
            n, P, T, m = self.systems[s]
            C = nm_matrix(P)
            p, F = self._view(self.p, s), self._view(self.F, s)
            p += (self.dt / 2) * F / MVV2E
            pt = np.einsum("jk,jnc->knc", C, p)
            pt = self._o_step(s, pt, self._view(xi1, s))
            p[...] = np.einsum("jk,knc->jnc", C, pt)
        self.step_count += 1

    # -- estimators (Sec. 2.1 finite-P average; Fig. S-beads virial KE) -------
    def estimators(self):
        out = []
        for s in range(len(self.systems)):
            n, P, T, m = self.systems[s]
            beta = 1.0 / (KB * T)
            _, wP = mode_frequencies(P, T)
            q, p, F = self._view(self.q, s), self._view(self.p, s), self._view(self.F, s)
            E = self.E[self._bead_slice(s)]
            dq = np.roll(q, -1, axis=0) - q
            e_spring = 0.5 * MVV2E * wP * wP * np.sum(m[None, :, None] * dq * dq) if P > 1 else 0.0
            qbar = q.mean(axis=0)
            k_beads = 0.5 * MVV2E * np.sum(p * p / m[None, :, None])
            v_sum = float(np.sum(E))
            k_cv = 3 * n / (2 * beta) - np.sum((q - qbar[None]) * F) / (2 * P)
            out.append(dict(
                V_bar=v_sum / P,
                K_prim=3 * n * P / (2 * beta) - e_spring / P,
                K_cv=k_cv,
                E_spring=e_spring,
                K_beads=k_beads,
                T_beads=2 * k_beads / (3 * n * P * KB),
                H_conserved=k_beads + e_spring + v_sum + self.heat[s],
                heat_bath=self.heat[s],
                P_cv=self._pressure_cv(s, k_cv)))
        return out

    def _pressure_cv(self, s, k_cv):
        """Centroid-virial pressure (eV/A^3) of a periodic system: scaling the
        box and the centroids by (1 + e) while the beads keep their offsets
        from their centroids leaves the springs unchanged, and
          P_cv = (2 K_cv + (1/P) sum_k tr W^(k)) / (3 V),
        with W^(k) the virial of bead k (W_ab = -dE/deps_ab); the offsets'
        share of tr W is the -(q - qbar).F term inside K_cv.  0 without a box
        or without bead virials."""
        if self.boxes is None or self.W is None or not np.all(self.boxes[s] > 0):
            return 0.0
        P = self.systems[s][1]
        trW = float(np.sum(np.trace(self.W[self._bead_slice(s)], axis1=1, axis2=2)))
        return (2.0 * k_cv + trW / P) / (3.0 * float(np.prod(self.boxes[s])))

    def _bead_slice(self, s):
        b0 = sum(P for _, P, _, _ in self.systems[:s])
        return slice(b0, b0 + self.systems[s][1])


# ---------------------------------------------------------------- staging
# Sec. 2.1 names the staging transformation beside normal modes as the way to
# decouple the ring-polymer springs (Tuckerman, Berne, Martyna, Klein, J.
# Chem. Phys. 99, 2796 (1993)).  With beads r_1..r_P (r_{P+1} = r_1):
#   u_1 = r_1,   u_l = r_l - ((l - 1) r_{l+1} + r_1) / l   (l = 2..P),
# the springs become sum_{l>=2} 1/2 m_l' w_P^2 u_l^2 with m_l' = l m / (l - 1).
# Kinetic masses: those of staging dynamics in the primitive form (V/P at
# beta: m~_1 = m, m~_l = m_l'), carried over to the bead-potential form used
# here (V at beta/P), which multiplies every kinetic mass by P:
# m~_1 = P m, m~_l = P m_l'.  Then u_1 carries the sum of the bead forces
# with P times the mass (physical time scales), and every u_l (l >= 2)
# oscillates at w_s = w_P / sqrt(P).  The momenta p~_l conjugate to u_l are
# the state; the thermostat is a Langevin friction per staging coordinate,
# gamma_1 = 1/tau0, gamma_l = 2 lambda w_s.  Arrays below are [P, ...] with
# index k = l - 1.


def staging_forward(r):
    """u from bead values r [P, ...]."""
    r = np.asarray(r, dtype=np.float64)
    P = len(r)
    u = np.empty_like(r)
    u[0] = r[0]
    for k in range(1, P):
        l = k + 1
        u[k] = r[k] - ((l - 1) * r[(k + 1) % P] + r[0]) / l
    return u


def staging_inverse(u):
    """r from u, by the recursion r_l = u_l + ((l - 1)/l) r_{l+1} + u_1 / l from l = P down."""
    u = np.asarray(u, dtype=np.float64)
    P = len(u)
    r = np.empty_like(u)
    r[0] = u[0]
    nxt = u[0]
    for k in range(P - 1, 0, -1):
        l = k + 1
        r[k] = u[k] + ((l - 1) / l) * nxt + u[0] / l
        nxt = r[k]
    return r


def staging_forces(F):
    """-dU/du from F = -dU/dr [P, ...]: the chain rule through r(u), summed as
    f~_1 = sum_l F_l,  f~_2 = F_2,  f~_l = F_l + ((l - 2)/(l - 1)) f~_{l-1}."""
    F = np.asarray(F, dtype=np.float64)
    P = len(F)
    G = np.empty_like(F)
    G[0] = F.sum(axis=0)
    for k in range(1, P):
        l = k + 1
        G[k] = F[k] + ((l - 2) / (l - 1)) * G[k - 1] if l > 2 else F[k]
    return G


def staging_mass_factors(P):
    """m_l' / m of the staging springs: l / (l - 1) for l >= 2 (1 for l = 1,
    which carries no spring)."""
    return np.array([1.0] + [(k + 1) / k for k in range(1, P)])


def staging_kinetic_factors(P):
    """m~_l / m = P m_l' / m (see above)."""
    return P * staging_mass_factors(P)


class StagingRingPolymers(RingPolymers):
    """RingPolymers propagated in staging coordinates (same splitting
    O(dt/2) B(dt/2) A(dt) [forces] B(dt/2) O(dt/2)).  The state momenta p are
    the staging momenta p~ (row of bead k holds p~ of staging coordinate k)."""

    def _o_step_staging(self, s, pt, xi):
        n, P, T, m = self.systems[s]
        _, wP = mode_frequencies(P, T)
        mt = staging_kinetic_factors(P)[:, None] * m[None, :]
        if self.tau0 > 0:
            gamma = np.full(P, 2.0 * self.lam * wP / np.sqrt(P))
            gamma[0] = 1.0 / self.tau0
        else:
            gamma = np.zeros(P)
        c1 = np.exp(-gamma * self.dt / 2)
        c2 = np.sqrt(1.0 - c1 * c1)
        sigma = np.sqrt(mt * KB * T * P / MVV2E)
        ke0 = 0.5 * MVV2E * np.sum(pt * pt / mt[:, :, None])
        pt = c1[:, None, None] * pt + sigma[:, :, None] * c2[:, None, None] * xi
        ke1 = 0.5 * MVV2E * np.sum(pt * pt / mt[:, :, None])
        self.heat[s] -= ke1 - ke0
        return pt

    def step(self, noise=None):
        xi0 = self._noise(0, noise)
        for s in range(len(self.systems)):
            n, P, T, m = self.systems[s]
            _, wP = mode_frequencies(P, T)
            ws = wP / np.sqrt(P)
            mt = staging_kinetic_factors(P)[:, None] * m[None, :]
            p, q, F = self._view(self.p, s), self._view(self.q, s), self._view(self.F, s)
            pt = self._o_step_staging(s, p.copy(), self._view(xi0, s))
            pt = pt + (self.dt / 2) * staging_forces(F) / MVV2E
            u = staging_forward(q)
            u[0] = u[0] + self.dt * pt[0] / mt[0][:, None]
            if P > 1:
                c, sn = np.cos(ws * self.dt), np.sin(ws * self.dt)
                mw = mt[1:, :, None] * ws
                un = sn * pt[1:] / mw + c * u[1:]
                pn = c * pt[1:] - mw * sn * u[1:]
                u[1:], pt[1:] = un, pn
            q[...] = staging_inverse(u)
            p[...] = pt
        self._forces()
        xi1 = self._noise(1, noise)
        for s in range(len(self.systems)):
            p, F = self._view(self.p, s), self._view(self.F, s)
            pt = p + (self.dt / 2) * staging_forces(F) / MVV2E
            p[...] = self._o_step_staging(s, pt, self._view(xi1, s))
        self.step_count += 1

    def estimators(self):
        out = super().estimators()
        for s, o in enumerate(out):
            n, P, T, m = self.systems[s]
            mt = staging_kinetic_factors(P)[:, None] * m[None, :]
            p = self._view(self.p, s)
            k_beads = 0.5 * MVV2E * np.sum(p * p / mt[:, :, None])
            o["H_conserved"] += k_beads - o["K_beads"]
            o["K_beads"] = k_beads
            o["T_beads"] = 2 * k_beads / (3 * n * P * KB)
        return out


# ---------------------------------------------------------------- primitive
# Sec. 2.3 also runs "primitive" PIMD: the inter-bead springs are one more
# force term and the beads move in Cartesian coordinates.  Here: the same
# O(dt/2) B(dt/2) A(dt) [forces] B(dt/2) O(dt/2) splitting with
#   B: p_k += dt/2 (F_k - m w_P^2 (2 q_k - q_{k+1} - q_{k-1})),
#   A: q_k += dt p_k / m (free drift),
#   O: Langevin friction 1/tau0 on every bead's momentum,
# i.e. velocity Verlet on the full ring Hamiltonian H_P; the spring
# frequencies up to 2 w_P must stay well below 2/dt.


def spring_forces(q, m, wP):
    """-dE_spring/dq of one system's beads q [P, n, 3] (eV/A), E_spring =
    sum_k 1/2 m w_P^2 |q_{k+1} - q_k|^2 (cyclic)."""
    if len(q) == 1:
        return np.zeros_like(q)
    lap = 2.0 * q - np.roll(q, -1, axis=0) - np.roll(q, 1, axis=0)
    return -(m[None, :, None] * wP * wP * MVV2E) * lap


class PrimitiveRingPolymers(RingPolymers):
    """RingPolymers propagated in Cartesian bead coordinates with the
    springs as forces (see above)."""

    def _o_step_beads(self, s, p, xi):
        n, P, T, m = self.systems[s]
        gamma = 1.0 / self.tau0 if self.tau0 > 0 else 0.0
        c1 = np.exp(-gamma * self.dt / 2)
        c2 = np.sqrt(1.0 - c1 * c1)
        sigma = np.sqrt(m * KB * T * P / MVV2E)
        ke0 = 0.5 * MVV2E * np.sum(p * p / m[None, :, None])
        p = c1 * p + sigma[None, :, None] * c2 * xi
        ke1 = 0.5 * MVV2E * np.sum(p * p / m[None, :, None])
        self.heat[s] -= ke1 - ke0
        return p

    def step(self, noise=None):
        xi0 = self._noise(0, noise)
        for s in range(len(self.systems)):
            n, P, T, m = self.systems[s]
            _, wP = mode_frequencies(P, T)
            p, q, F = self._view(self.p, s), self._view(self.q, s), self._view(self.F, s)
            pt = self._o_step_beads(s, p.copy(), self._view(xi0, s))
            pt = pt + (self.dt / 2) * (F + spring_forces(q, m, wP)) / MVV2E
            q[...] = q + self.dt * pt / m[None, :, None]
            p[...] = pt
        self._forces()
        xi1 = self._noise(1, noise)
        for s in range(len(self.systems)):
            n, P, T, m = self.systems[s]
            _, wP = mode_frequencies(P, T)
            p, q, F = self._view(self.p, s), self._view(self.q, s), self._view(self.F, s)
            pt = p + (self.dt / 2) * (F + spring_forces(q, m, wP)) / MVV2E
            p[...] = self._o_step_beads(s, pt, self._view(xi1, s))
        self.step_count += 1


def harmonic_force_fn(systems, omega):
    """V = sum_i 1/2 m_i omega^2 |q_i|^2 per bead (isotropic oscillator about
    the origin); returns E per bead and F = -m omega^2 q."""
    masses = np.concatenate([np.tile(m, P) for n, P, _, m in systems])
    bead_off = np.cumsum([0] + [P for _, P, _, _ in systems])
    bead_id = np.concatenate([bead_off[s] + np.repeat(np.arange(P), n)
                              for s, (n, P, _, _) in enumerate(systems)])

    def fn(q):
        k = masses * omega * omega * MVV2E
        e_atom = 0.5 * k * np.sum(q * q, axis=1)
        E = np.bincount(bead_id, weights=e_atom, minlength=int(bead_off[-1]))
        return E, -k[:, None] * q
    return fn
