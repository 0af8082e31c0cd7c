"""Ground-truth MB positions in plane pixel coordinates (training labels and
evaluation truth).

Orientation 0 images the x-z plane (u = x), orientation 1 the y-z plane
(u = y); pixel coordinates have pixel centres at integers:
    z_pix = (z - z0) / dz,   u_pix = (u - u0) / du.
With B slabs along v, an MB belongs to the slab whose v range holds it.
"""
from __future__ import annotations

import numpy as np

from .configs import Config
from .medium import Medium


def plane_positions(cfg: Config, medium: Medium, margin: float = 0.5):
    """For every plane p = o * B + b and frame f: array [n][2] of (z_pix, u_pix) of
    the MBs inside the grid (extended by `margin` pixels).  Returns a list over
    planes of lists over frames."""
    g = cfg.grid
    mb = medium.mb_positions()                       # [F][M][3] (x, y, z)
    per = -(-g.nv // g.n_blocks)
    out = []
    for o in range(2):
        u = mb[..., 0] if o == 0 else mb[..., 1]
        v = mb[..., 1] if o == 0 else mb[..., 0]
        zp = (mb[..., 2] - g.z0) / g.dz
        up = (u - g.u0) / g.du
        vp = np.rint((v - g.v0) / g.dv)
        inside = (zp >= -margin) & (zp <= g.nz - 1 + margin) & (up >= -margin) & \
                 (up <= g.nu - 1 + margin)
        for b in range(g.n_blocks):
            lo, hi = b * per, min(g.nv, (b + 1) * per)
            sel = inside & (vp >= lo) & (vp < hi) if g.n_blocks > 1 else inside
            out.append([np.stack([zp[f][sel[f]], up[f][sel[f]]], axis=1)
                        for f in range(mb.shape[0])])
    return out
