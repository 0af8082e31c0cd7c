"""Seeded localisation lists of the two orthogonal planes, for the pairing
tests: 3D MB positions per frame seen by both projections with small position
and intensity jitter, plus unpaired records (an MB seen by one plane only).

Records carry the fields of a localisation record (plane, frame, iz, iu, z, u,
ncc, intensity) with plane = orientation * n_blocks + slab, the slab being the
index of the projected-out coordinate's slab (y for the XZ plane, x for YZ),
and are sorted by (plane, frame, iz, iu) like the localisers' output."""
from __future__ import annotations

import numpy as np

RECORD_DTYPE = np.dtype([("plane", np.int32), ("frame", np.int32), ("iz", np.int32),
                         ("iu", np.int32), ("z", np.float32), ("u", np.float32),
                         ("ncc", np.float32), ("intensity", np.float32)])


def plane_records(nz: int, nv: int, n_blocks: int, n_frames: int, mb_per_frame: int, seed: int,
                  pos_sigma: float = 0.25, int_sigma: float = 0.02, single_frac: float = 0.2):
    """Returns (records, truth): records as above; truth[f] = [M][4] (x, y, z,
    intensity) of the MBs of frame f.  x, y in [0, nv), z in [0, nz) plane
    pixels; intensities log-uniform over a decade."""
    g = np.random.default_rng(seed)
    per = -(-nv // n_blocks)
    rows, truth = [], []
    for f in range(n_frames):
        m = int(g.poisson(mb_per_frame)) if mb_per_frame > 0 else 0
        x = g.uniform(0, nv - 1, m)
        y = g.uniform(0, nv - 1, m)
        z = g.uniform(0, nz - 1, m)
        inten = np.exp(g.uniform(np.log(0.1), np.log(1.0), m))
        truth.append(np.stack([x, y, z, inten], axis=1) if m else np.zeros((0, 4)))
        seen_xz = g.uniform(size=m) >= single_frac / 2
        seen_yz = g.uniform(size=m) >= single_frac / 2
        for o, (u, other, seen) in enumerate(((x, y, seen_xz), (y, x, seen_yz))):
            for k in np.nonzero(seen)[0]:
                zz = z[k] + g.normal(0, pos_sigma)
                uu = u[k] + g.normal(0, pos_sigma)
                ii = inten[k] * (1.0 + g.normal(0, int_sigma))
                slab = min(int(np.floor(other[k] + 0.5)) // per, n_blocks - 1) if n_blocks > 1 else 0
                rows.append((o * n_blocks + slab, f, int(np.floor(zz + 0.5)), int(np.floor(uu + 0.5)),
                             zz, uu, 0.9, ii))
    rec = np.array(rows, dtype=RECORD_DTYPE) if rows else np.zeros(0, RECORD_DTYPE)
    order = np.lexsort((rec["iu"], rec["iz"], rec["frame"], rec["plane"]))
    return rec[order], truth
