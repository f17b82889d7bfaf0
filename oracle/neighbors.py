"""Neighbour sets under the cutoff (oracle side).

Definition: N(i) = { j != i : |d_ij| < R_c }, d_ij the minimum-image vector
q_j - q_i for a periodic orthorhombic box (raw difference otherwise); the
molecular graph of the paper (Sec. 2.2) with the 0.6 nm cutoff of Tables
S1/S2.  The cutoff must be below half of every box length, so one image per
pair exists.

Membership is decided in float32 with this operation order, one rounding per
operation and no fused multiply-add (numpy float32 arrays never fuse):
  x_w = x - L floor(x invL),   invL = fl32(1/L)           (wrap into the box)
  d   = x_w[j] - x_w[i];  d -= L rint(d invL)             (minimum image)
  r2  = (dx dx + dy dy) + dz dz;  include iff r2 < fl32(R_c^2)
Lists are sorted by (i, j).  `fp64_pairs` gives the FP64 set for comparison;
the two may only differ for pairs with |r^2 - R_c^2| < 1e-4 A^2.
"""
import numpy as np


def _wrap32(q32, box):
    L = box.astype(np.float32)
    invL = (1.0 / box).astype(np.float32)
    return q32 - L * np.floor(q32 * invL)


def _pair_r2_32(xw, rows, box, periodic):
    d = xw[None, :, :] - xw[rows, None, :]
    if periodic:
        L = box.astype(np.float32)
        invL = (1.0 / box).astype(np.float32)
        d = d - L * np.rint(d * invL)
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def brute_force_fp32(q32, box, cutoff, chunk=512):
    """CSR (start[int64 n+1], idx[int32]) of the float32 neighbour sets of one bead."""
    q32 = np.asarray(q32, dtype=np.float32)
    box = np.asarray(box, dtype=np.float64)
    periodic = bool(np.any(box > 0))
    n = len(q32)
    if periodic and not np.all(cutoff < 0.5 * box):
        raise ValueError("cutoff must be below half of every box length")
    xw = _wrap32(q32, box) if periodic else q32
    rc2 = np.float32(cutoff * cutoff)
    counts = np.zeros(n, dtype=np.int64)
    parts = []
    for lo in range(0, n, chunk):
        rows = np.arange(lo, min(n, lo + chunk))
        r2 = _pair_r2_32(xw, rows, box, periodic)
        mask = r2 < rc2
        mask[np.arange(len(rows)), rows] = False
        counts[rows] = mask.sum(axis=1)
        parts.append(np.nonzero(mask)[1].astype(np.int32))
    start = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=start[1:])
    return start, (np.concatenate(parts) if parts else np.zeros(0, np.int32))


def cell_list_fp32(q32, box, cutoff):
    """Same sets through a cell list: cells of width >= R_c, each atom scans its
    own and the adjacent cells (the stencil collapses to all cells along an
    axis with fewer than 3 cells, each cell taken once)."""
    q32 = np.asarray(q32, dtype=np.float32)
    box = np.asarray(box, dtype=np.float64)
    n = len(q32)
    xw = _wrap32(q32, box)
    nc = np.maximum(1, np.floor(box / (cutoff + 1e-4)).astype(int))
    cell = np.minimum((xw.astype(np.float64) / box * nc).astype(int), nc - 1)
    members = {}
    for a, c in enumerate(map(tuple, cell)):
        members.setdefault(c, []).append(a)
    rc2 = np.float32(cutoff * cutoff)
    L = box.astype(np.float32)
    invL = (1.0 / box).astype(np.float32)
    lists = []
    for i in range(n):
        axes = []
        for dim in range(3):
            if nc[dim] < 3:
                axes.append(range(nc[dim]))
            else:
                axes.append(sorted({(cell[i, dim] + o) % nc[dim] for o in (-1, 0, 1)}))
        cand = []
        for cx in axes[0]:
            for cy in axes[1]:
                for cz in axes[2]:
                    cand.extend(members.get((cx, cy, cz), []))
        cand = np.array(sorted(cand), dtype=np.int64)
        d = xw[cand] - xw[i]
        d = d - L * np.rint(d * invL)
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        keep = (r2 < rc2) & (cand != i)
        lists.append(cand[keep].astype(np.int32))
    start = np.zeros(n + 1, dtype=np.int64)
    np.cumsum([len(x) for x in lists], out=start[1:])
    return start, (np.concatenate(lists) if lists else np.zeros(0, np.int32))


def fp64_pairs(q, box, cutoff):
    """FP64 neighbour set as a boolean matrix and the matrix of r^2."""
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    d = q[None, :, :] - q[:, None, :]
    if np.any(box > 0):
        d = d - box * np.round(d / box)
    r2 = np.einsum("ijk,ijk->ij", d, d)
    mask = r2 < cutoff * cutoff
    np.fill_diagonal(mask, False)
    return mask, r2


def csr_to_dense(start, idx, n):
    m = np.zeros((n, n), dtype=bool)
    for i in range(n):
        m[i, idx[start[i]:start[i + 1]]] = True
    return m
