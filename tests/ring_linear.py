"""Exact stationary statistics of one thermostatted ring-polymer step in a
harmonic well (test helper, Sec. S1 protocol).

With a harmonic potential, one O B A B O step is an affine map of the state
and the two noise draws: z' = A z + B xi, with z the x components of the P
bead positions followed by the P bead momenta of one atom (the y and z
components are independent copies).  A and B are read off the integrator
itself as black boxes: one step of 2P independent atoms, atom a starting at
unit vector a with no noise, gives the columns of A; one step of 2P atoms at
rest, atom a receiving unit noise a, gives the columns of B.  The chain's
stationary covariance then solves Sigma = A Sigma A^T + B B^T.  Its bead
position variance is the average the thermostat samples, without sampling
error, and quadratic estimators are averaged exactly over Sigma.
"""
import numpy as np
from scipy.linalg import cholesky, solve_discrete_lyapunov


def step_maps(one_step, P):
    """one_step(q[P*n, 3], p[P*n, 3], xi[2, P*n, 3]) -> (q', p') for n = 2P
    independent atoms in the bead-major layout (index = k n + i).  Returns
    (A, B), both 2P x 2P."""
    n = 2 * P
    q = np.zeros((P, n, 3))
    p = np.zeros((P, n, 3))
    for a in range(P):
        q[a, a, 0] = 1.0
        p[a, P + a, 0] = 1.0
    q1, p1 = one_step(q.reshape(-1, 3), p.reshape(-1, 3), np.zeros((2, P * n, 3)))
    q1, p1 = np.asarray(q1, np.float64).reshape(P, n, 3), np.asarray(p1, np.float64).reshape(P, n, 3)
    A = np.concatenate([q1[:, :, 0], p1[:, :, 0]], axis=0)
    xi = np.zeros((2, P, n, 3))
    for a in range(2 * P):
        xi[a // P, a % P, a, 0] = 1.0
    z = np.zeros((P * n, 3))
    q2, p2 = one_step(z, z, xi.reshape(2, P * n, 3))
    q2, p2 = np.asarray(q2, np.float64).reshape(P, n, 3), np.asarray(p2, np.float64).reshape(P, n, 3)
    B = np.concatenate([q2[:, :, 0], p2[:, :, 0]], axis=0)
    return A, B


def stationary_covariance(A, B):
    S = solve_discrete_lyapunov(A, B @ B.T)
    return 0.5 * (S + S.T)


def bead_x2(S, P):
    """Stationary <x^2> of a bead (every bead has the same variance)."""
    return float(np.mean(np.diag(S)[:P]))


def quadratic_mean(estimate, S, P):
    """Exact mean over N(0, S) (every Cartesian component an independent copy)
    of an estimator that is a constant plus a quadratic form of one atom's
    bead positions: estimate(q[P, 3]) -> float.  Positions only: the
    momentum block of S is not used."""
    L = cholesky(S[:P, :P] + 1e-300 * np.eye(P), lower=True)
    zero = np.zeros((P, 3))
    c = estimate(zero)
    total = c
    for i in range(P):
        for comp in range(3):
            q = np.zeros((P, 3))
            q[:, comp] = L[:, i]
            total += estimate(q) - c
    return total
