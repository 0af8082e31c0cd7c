"""Oracle: pairing of the two orthogonal projections' 2D localisations into 3D
MB positions (CPU).

TEST INFRASTRUCTURE ONLY.

The paper's projection-based 3D localisation (Section II-A4): XZ localisations
(the x-z plane) and YZ localisations (the y-z plane) of the same frame are
paired.  For an XZ localisation i, every YZ localisation j within one voxel
axially, |z_i - z_j| <= 1 (plane pixel units), is a candidate; a candidate is
kept only if the intensity ratio rho = I_i / I_j lies in [0.9, 1.11].  Final
pairs are the mutual minima: j is i's best candidate and i is j's best
candidate.  The 3D position takes x from the XZ localisation, y from the YZ
localisation and the mean of the two z.

Readings (the paper gives only the rule in words):
  * "minimum intensity ratio" is taken as the ratio closest to 1, measured by
    max(rho, 1/rho); ties go to the smaller index;
  * with the plane split into B slabs, an XZ localisation of slab b (slab of
    y) pairs only with YZ localisations whose y lies in slab b, and its x must
    lie in the YZ localisation's slab (slab of x);
  * the ratio gate, the closeness and the axial test are decided in FP32 (the
    precision of the localisation records).
"""
from __future__ import annotations

import numpy as np

RATIO_LO = np.float32(0.9)
RATIO_HI = np.float32(1.11)


def _slab(pix, per):
    """Slab of a plane coordinate: its nearest pixel (the half-way shift taken
    in FP32, like the records) over the slab width; -1 below pixel 0."""
    r = np.floor(np.asarray(pix, np.float32) + np.float32(0.5)).astype(np.float64)
    with np.errstate(invalid="ignore"):
        s = np.where(np.isfinite(r) & (r >= 0) & (r < 1e6), r, -per) // per
    return s.astype(np.int64)


def _cost_rows(xz, yz, rows, per):
    """Cost of pairing XZ records `rows` with every YZ record: max(rho, 1/rho)
    for candidates, +inf otherwise (FP32)."""
    zi = xz["z"][rows].astype(np.float32)[:, None]
    zj = yz["z"].astype(np.float32)[None, :]
    Ii = xz["intensity"][rows].astype(np.float32)[:, None]
    Ij = yz["intensity"].astype(np.float32)[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        rho = (Ii / Ij).astype(np.float32)
        inv = (Ij / Ii).astype(np.float32)
    ok = (np.abs(zi - zj) <= np.float32(1.0)) & (rho >= RATIO_LO) & (rho <= RATIO_HI)
    ok &= (Ii > 0) & (Ij > 0)
    if per is not None:
        # slab consistency: y of the YZ record in the XZ record's slab, and vice versa
        ok &= _slab(yz["u"], per)[None, :] == xz["block"][rows][:, None]
        ok &= _slab(xz["u"][rows], per)[:, None] == yz["block"][None, :]
    return np.where(ok, np.maximum(rho, inv), np.float32(np.inf)).astype(np.float32)


def pair_frame(xz, yz, per=None, chunk=1024):
    """xz, yz: arrays with fields z, u, intensity (float32) and block.  Returns
    a list of (i, j) index pairs in increasing i.  The cost matrix is formed
    `chunk` XZ rows at a time; every record's best candidate is the first
    minimum in index order."""
    n, m = len(xz), len(yz)
    if n == 0 or m == 0:
        return []
    best_j = np.full(n, -1)
    col_min = np.full(m, np.float32(np.inf), dtype=np.float32)
    best_i = np.full(m, -1)
    for r0 in range(0, n, chunk):
        rows = np.arange(r0, min(n, r0 + chunk))
        cost = _cost_rows(xz, yz, rows, per)
        for a, i in enumerate(rows):
            if np.isfinite(cost[a]).any():
                best_j[i] = int(np.argmin(cost[a]))          # first minimum = smaller index
        cm = cost.min(axis=0)
        ca = rows[0] + np.argmin(cost, axis=0)               # first row reaching the chunk's minimum
        upd = cm < col_min                                   # strict: earlier chunks keep ties
        col_min = np.where(upd, cm, col_min)
        best_i = np.where(upd & np.isfinite(cm), ca, best_i)
    return [(i, int(best_j[i])) for i in range(n) if best_j[i] >= 0 and best_i[best_j[i]] == i]


def pair_localisations(locs, n_blocks: int, nv: int, frames=None):
    """locs: records (plane, frame, z, u, intensity) of both orientations, plane =
    o * n_blocks + b.  Returns a structured array of 3D localisations sorted by
    (frame, XZ record index): frame, x, y, z (plane pixels), the two
    intensities and the indices of the paired records in `locs`.  `frames`
    limits the pairing to those frames (frames are paired independently)."""
    out = []
    per = -(-nv // n_blocks)
    locs = np.asarray(locs)
    idx = np.arange(len(locs))
    todo = np.unique(locs["frame"]) if len(locs) else []
    if frames is not None:
        todo = [f for f in todo if f in set(int(x) for x in frames)]
    for f in todo:
        sel = locs["frame"] == f
        a_mask = sel & (locs["plane"] < n_blocks)
        b_mask = sel & (locs["plane"] >= n_blocks)
        A, B = locs[a_mask], locs[b_mask]
        ia, ib = idx[a_mask], idx[b_mask]
        xz = np.zeros(len(A), dtype=[("z", "f4"), ("u", "f4"), ("intensity", "f4"), ("block", "i8")])
        yz = np.zeros(len(B), dtype=xz.dtype)
        for dst, src, o in ((xz, A, 0), (yz, B, 1)):
            dst["z"], dst["u"], dst["intensity"] = src["z"], src["u"], src["intensity"]
            dst["block"] = src["plane"] - o * n_blocks
        for i, j in pair_frame(xz, yz, per if n_blocks > 1 else None):
            z = (np.float32(xz["z"][i]) + np.float32(yz["z"][j])) * np.float32(0.5)
            out.append((int(f), float(xz["u"][i]), float(yz["u"][j]), float(z),
                        float(xz["intensity"][i]), float(yz["intensity"][j]), int(ia[i]), int(ib[j])))
    return np.array(out, dtype=LOC3D_DTYPE)


LOC3D_DTYPE = np.dtype([("frame", np.int32), ("x", np.float32), ("y", np.float32),
                        ("z", np.float32), ("i_xz", np.float32), ("i_yz", np.float32),
                        ("idx_xz", np.int32), ("idx_yz", np.int32)])
