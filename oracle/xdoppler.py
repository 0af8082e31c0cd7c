"""Oracle: XDoppler of the projection planes (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

Section II-A4: beamforming, clutter filtering and separation are applied to
the RC and CR volumes separately, and the filtered RC and CR stacks are
cross-correlated with a window of three frames (the XDoppler scheme, which the
paper cites and does not print) before localisation.  In the projection form
the two orientations' planes are different planes (x-z for RC, y-z for CR), so
the reading taken here is:

  * Both orientations' compounded volumes live on one voxel grid (x, y, z).
    Each plane (orientation o, slab b) therefore has two stacks: its own
    orientation's volume sum-projected over the slab (P, what the two-stage
    beamformer already forms) and the other orientation's volume
    sum-projected over the same slab onto the same plane (the cross
    projection Q).  For the x-z plane of slab b:
        P_{0,b}(x, z) = sum_{y in b} V_RC(u = x, v = y, z)
        Q_{0,b}(x, z) = sum_{y in b} V_CR(u = y, v = x, z)
    and for the y-z plane the roles of RC and CR swap.  V is stage 2's
    volume (every slice the reference slice moved by the rigid axial shift,
    compounded over the transmits).  The plane's lateral axis is the other
    orientation's v axis, so the cross projection needs the v grid to equal
    the u grid.
  * P and Q are clutter-filtered separately.  The XDoppler value of frame f is
    their zero-lag cross-correlation over the frames f - h .. f + h that exist
    (h = (window - 1) / 2):  X_f = sum_t P_t conj(Q_t).
  * Localisation runs on sqrt(|X_f|): for one MB with amplitudes a (RC) and b
    (CR) that is the geometric mean of the two, so a Gaussian PSF keeps its
    width and the localiser's template applies unchanged.  The image is
    returned as a complex stack with zero imaginary part, whose envelope is
    sqrt(|X_f|).
"""
from __future__ import annotations

import numpy as np

from .beamform import block_ranges


def cross_project(S, cfg) -> np.ndarray:
    """Cross projections Q[o][b][f][z][i] from the stage-1 slices S[o][k][f][z][u].

    Plane o receives the other orientation o' = 1 - o: its volume's slice at
    v = v_i (v_i = v0 + i dv, the plane's lateral coordinate) is built from the
    reference slice as in stage 2 and summed over the u samples of block b.
    The volume is built slice by slice, literally.
    """
    g = cfg.grid
    O, K, F, nz, nu = S.shape
    if g.nv != nu or g.dv != g.du or g.v0 != g.u0:
        raise ValueError("the cross projection needs the v grid to equal the u grid")
    out = np.zeros((O, g.n_blocks, F, nz, g.nv), dtype=np.complex128)
    ang = np.asarray(cfg.seq.angles_rad)
    blocks = block_ranges(cfg)
    for o in range(O):
        src = S[1 - o]
        for k in range(K):
            t = np.tan(ang[k] / 2.0)
            for i in range(g.nv):
                v = g.v0 + i * g.dv
                dz_m = (v - g.v_ref) * t
                shift = dz_m / g.dz
                phase = np.exp(1j * 4.0 * np.pi * cfg.probe.f0 * dz_m / cfg.probe.c)
                # the volume's slice at v: S^lin(u, z + shift) for every u
                sl = np.zeros((F, nz, nu), dtype=np.complex128)
                n_int = int(np.floor(shift))
                fr = shift - n_int
                for (w, off) in ((1.0 - fr, n_int), (fr, n_int + 1)):
                    if w == 0.0:
                        continue
                    l_lo, l_hi = max(0, -off), min(nz, nz - off)
                    if l_hi > l_lo:
                        sl[:, l_lo:l_hi, :] += w * src[k, :, l_lo + off:l_hi + off, :]
                for b, (m_lo, m_hi) in enumerate(blocks):
                    out[o, b, :, :, i] += phase * sl[:, :, m_lo:m_hi].sum(axis=2)
    return out


def xdoppler(P, Q, window: int = 3) -> np.ndarray:
    """sqrt(|sum_{t in W(f)} P_t conj(Q_t)|) per pixel, W(f) = frames f - h .. f + h
    inside the ensemble; P, Q: [O][B][F][z][u].  Returns complex128 (zero
    imaginary part), the image the localiser takes."""
    P = np.asarray(P, dtype=np.complex128)
    Q = np.asarray(Q, dtype=np.complex128)
    if window < 1 or window % 2 == 0:
        raise ValueError("window must be odd and positive")
    h = (window - 1) // 2
    F = P.shape[2]
    prod = P * np.conj(Q)
    out = np.zeros(P.shape, dtype=np.complex128)
    for f in range(F):
        x = prod[:, :, max(0, f - h):min(F, f + h + 1)].sum(axis=2)
        out[:, :, f] = np.sqrt(np.abs(x))
    return out
