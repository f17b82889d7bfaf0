"""Direct-force head in the form of the paper's graph field network (FP64,
oracle side; test infrastructure only).

Sec. 2.2 treats forces as an edge property: messages from edges update the
nodes, the two end nodes update each edge, and the force on i is a sum of
edge terms along the edge directions.  Written out for the synthetic head
(every reading below is stated in the design notes):

  rho_s(r)   = exp(-eta_s (r - R_s)^2) f_c(r),  f_c(r) = (cos(pi r / r_c) + 1) / 2
  n_i^(0)    = a[Z_i]
  e_ij^(0)   = W_r rho(r_ij) + b[Z_i, Z_j]                  (b symmetric)
  m_i^(l)    = sum_{j in N(i)} phi_m^(l)(e_ij^(l))           (messages summed over the edges)
  n_i^(l+1)  = n_i^(l) + phi_v^(l)([n_i^(l); m_i^(l)])
  e_ij^(l+1) = e_ij^(l) + phi_e^(l)(n_i^(l) + n_j^(l))       (symmetric aggregation of the end nodes)
  F_i        = sum_{j in N(i)} f_c(r_ij) u_ij phi_f(e_ij^(L)),  u_ij = (q_j - q_i) / r_ij

with phi(x) = W2 tanh(W1 x + b1) + b2 and phi_f(e) = w2 . tanh(W1 e + b1) + b2.
e_ij = e_ji and u_ij = -u_ji, so the edge forces obey Newton's third law.
There is no energy.
"""
import numpy as np

from . import neighbors


def _mlp(p, x):
    W1, b1, W2, b2 = (np.asarray(a, dtype=np.float64) for a in p)
    return np.tanh(x @ W1.T + b1) @ W2.T + b2


def edges(model, q32_bead, box):
    """Directed edges (owner i, neighbour j) of one bead, the FP64
    displacements d_ij and distances."""
    q32_bead = np.asarray(q32_bead, dtype=np.float32)
    start, idx = neighbors.brute_force_fp32(q32_bead, box, model.cutoff)
    q = q32_bead.astype(np.float64)
    owner = np.repeat(np.arange(len(q)), np.diff(start))
    d = q[idx] - q[owner]
    box = np.asarray(box, dtype=np.float64)
    if np.any(box > 0):
        d = d - box * np.round(d / box)
    return owner, idx.astype(np.int64), d, np.sqrt((d * d).sum(axis=1))


def edge_basis(model, r):
    """rho_s(r) [E, n_rad] and f_c(r) [E]."""
    fc = 0.5 * (np.cos(np.pi * r / model.cutoff) + 1.0)
    x = r[:, None] - np.asarray(model.rad_center)[None, :]
    return np.exp(-np.asarray(model.rad_eta)[None, :] * x * x) * fc[:, None], fc


def bead_forces(model, q32_bead, species, box, return_parts=False):
    """Forces [N, 3] (eV/A) of one bead from the head, in FP64."""
    species = np.asarray(species)
    n = len(species)
    owner, nbr, d, r = edges(model, q32_bead, box)
    rho, fc = edge_basis(model, r)
    e = rho @ np.asarray(model.edge_in, dtype=np.float64).T
    e = e + np.asarray(model.pair_embed, dtype=np.float64)[species[owner], species[nbr]]
    node = np.asarray(model.node_embed, dtype=np.float64)[species]
    nodes = [node]
    for msg, upd, edg in model.layers:
        m = np.zeros_like(node)
        np.add.at(m, owner, _mlp(msg, e))
        e = e + _mlp(edg, node[owner] + node[nbr])
        node = node + _mlp(upd, np.concatenate([node, m], axis=1))
        nodes.append(node)
    W1, b1, w2, b2 = (np.asarray(a, dtype=np.float64) for a in model.force)
    s = np.tanh(e @ W1.T + b1) @ w2 + b2
    F = np.zeros((n, 3))
    np.add.at(F, owner, (fc * s / r)[:, None] * d)
    if return_parts:
        return F, dict(owner=owner, nbr=nbr, d=d, r=r, e=e, s=s, nodes=nodes)
    return F


def forces(wl, q32):
    """All beads of all systems of a workload: F[sum P_s N_s, 3]."""
    q32 = np.asarray(q32, dtype=np.float32).reshape(-1, 3)
    out, off = [], 0
    for s in wl.systems:
        for _ in range(s.n_beads):
            out.append(bead_forces(wl.model, q32[off:off + s.n_atoms], s.species, s.box))
            off += s.n_atoms
    return np.concatenate(out)
