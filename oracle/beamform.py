"""Oracle: two-stage row-column beamforming to projection planes (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

Follows the paper's Section II-A1 (beamforming) and Section II-A4 (sub-block
sum projection):
  1. Stage 1 beamforms, for each transmit k of each orientation, one reference
     slice S_k(u, z) at v = v_ref from the channel data.
  2. Stage 2 extrapolates the volume V_k(u, v, z) from S_k along the transmit
     direction: every slice is the reference slice moved by a rigid axial shift
     that depends on the steering angle.
  3. The volumes of all transmits are summed coherently and the slices of each
     block along v are sum-projected onto one plane.

Stage 2's shift law is not printed in the paper (it cites earlier work).  The
reading used here: with a plane wave steered by theta in the v-z plane and the
paraxial receive delay, a scatterer seen at depth z in slice v appears in the
reference slice at depth z + (v - v_ref) * t, t = sin(theta)/(1 + cos(theta))
= tan(theta/2); in baseband the sample also turns by exp(+i 4 pi f0 (v - v_ref)
t / c).  The reference slice is linearly interpolated along z and is zero
outside the grid.
"""
from __future__ import annotations

import numpy as np

from . import _clib


def _probe(cfg):
    p = _clib.Probe()
    p.n_elem = cfg.probe.n_elem
    p.pitch = cfg.probe.pitch
    p.c = cfg.probe.c
    p.f0 = cfg.probe.f0
    p.fs = cfg.probe.fs
    p.t_start = cfg.seq.t_start
    p.n_samp = cfg.seq.n_samp
    return p


def _as_iq(iq, cfg):
    iq = np.ascontiguousarray(iq, dtype=np.complex128)
    F = iq.shape[0]
    if iq.shape[1:] != cfg.iq_shape[1:]:
        raise ValueError(f"iq shape {iq.shape} does not match {cfg.iq_shape}")
    return iq, F


def stage1_slices(iq, cfg) -> np.ndarray:
    """Stage-1 reference slices S[o][k][f][z][u] (complex128).

    iq: [F][O][K][Nc][Ns] complex.  Section II-A1, stage 1.
    """
    iq, F = _as_iq(iq, cfg)
    g = cfg.grid
    K = cfg.n_angles
    out = np.zeros((2, K, F, g.nz, g.nu), dtype=np.complex128)
    angles = np.ascontiguousarray(cfg.seq.angles_rad, dtype=np.float64)
    pr = _probe(cfg)
    _clib.lib().oracle_das_stage1(_clib.dptr(iq.view(np.float64)), F, 2, K, _clib.dptr(angles),
                                  pr, g.nu, g.nz, g.u0, g.du, g.z0, g.dz, g.v_ref,
                                  _clib.dptr(out.view(np.float64)))
    return out


def block_ranges(cfg):
    """Slice-index ranges [m_lo, m_hi) of the B blocks along v (equal split, last ragged)."""
    g = cfg.grid
    per = -(-g.nv // g.n_blocks)
    return [(b * per, min((b + 1) * per, g.nv)) for b in range(g.n_blocks)]


def stage2_project(S, cfg) -> np.ndarray:
    """Stage 2 plus compounding plus block sum-projection.

    S: [O][K][F][Nz][Nu] reference slices.  Returns P[o][b][f][z][u]:
        P_{o,b}(u, z) = sum_k sum_{m in b} V_k(u, v_m, z)
        V_k(u, v, z)  = S_k^lin(u, z + (v - v_ref) t_k) * exp(i 4 pi f0 (v - v_ref) t_k / c)
    The volume is extrapolated slice by slice (literally) and summed.
    """
    g = cfg.grid
    O, K, F, nz, nu = S.shape
    out = np.zeros((O, g.n_blocks, F, nz, nu), dtype=np.complex128)
    ang = np.asarray(cfg.seq.angles_rad)
    for b, (m_lo, m_hi) in enumerate(block_ranges(cfg)):
        for k in range(K):
            t = np.tan(ang[k] / 2.0)
            for m in range(m_lo, m_hi):
                v = g.v0 + m * g.dv
                dz_m = (v - g.v_ref) * t               # metres
                shift = dz_m / g.dz                    # pixels
                phase = np.exp(1j * 4.0 * np.pi * cfg.probe.f0 * dz_m / cfg.probe.c)
                # S^lin at row l + shift: (1 - fr) S[n0] + fr S[n0 + 1], zero outside [0, nz)
                n_int = int(np.floor(shift))
                fr = shift - n_int
                for (w, off) in ((1.0 - fr, n_int), (fr, n_int + 1)):
                    if w == 0.0:
                        continue
                    l_lo = max(0, -off)
                    l_hi = min(nz, nz - off)
                    if l_hi <= l_lo:
                        continue
                    out[:, b, :, l_lo:l_hi, :] += (w * phase) * S[:, k, :, l_lo + off:l_hi + off, :]
    return out


def beamform_proj(iq, cfg) -> np.ndarray:
    """Channel data -> projection planes P[o][b][f][z][u] (complex128)."""
    return stage2_project(stage1_slices(iq, cfg), cfg)


def das_3d_slab(iq, cfg, m_lo: int, m_hi: int) -> np.ndarray:
    """Conventional full-3D DAS of every voxel of slices [m_lo, m_hi) along v,
    sum-projected over those slices, kept per transmit: [O][K][F][Nz][Nu]."""
    iq, F = _as_iq(iq, cfg)
    g = cfg.grid
    K = cfg.n_angles
    out = np.zeros((2, K, F, g.nz, g.nu), dtype=np.complex128)
    angles = np.ascontiguousarray(cfg.seq.angles_rad, dtype=np.float64)
    pr = _probe(cfg)
    _clib.lib().oracle_das_3d_slab(_clib.dptr(iq.view(np.float64)), F, 2, K, _clib.dptr(angles),
                                   pr, g.nu, g.nz, g.u0, g.du, g.z0, g.dz, g.v0, g.dv,
                                   int(m_lo), int(m_hi), _clib.dptr(out.view(np.float64)))
    return out


def stage2_project_per_transmit(S, cfg, m_lo: int, m_hi: int) -> np.ndarray:
    """Stage 2 summed over slices [m_lo, m_hi) but kept per transmit:
    [O][K][F][Nz][Nu].  Used to compare with das_3d_slab transmit by transmit."""
    from dataclasses import replace
    O, K, F, nz, nu = S.shape
    out = np.zeros((O, K, F, nz, nu), dtype=np.complex128)
    for k in range(K):
        sub = cfg.with_(seq=replace(cfg.seq, angles_deg=(cfg.seq.angles_deg[k],)),
                        grid=replace(cfg.grid, n_blocks=1, v0=cfg.grid.v0 + m_lo * cfg.grid.dv,
                                     nv=m_hi - m_lo))
        out[:, k] = stage2_project(S[:, k:k + 1], sub)[:, 0]
    return out
