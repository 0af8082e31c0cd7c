"""Oracle: linear Gaussian-pulse forward model of RCA plane-wave channel data (FP64).

TEST INFRASTRUCTURE ONLY.

The paper's data (in-vivo pig kidney, phantoms, Field II simulations) is not
available, so inputs come from a forward model of the same acquisition
(Section II-C: row-column array, steered plane waves, IQ channel data):

  IQ_{f,o,k,e}(t_s) = sum_scatterers A * exp(-(t_s - tau)^2 / (2 sigma_t^2))
                                       * exp(-i 2 pi f0 tau)  +  noise
  t_s = t_start + s / fs
  tau = tau_tx(v, z; theta_k) + tau_rx(u, z; e)  with (u, v) = (x, y) for
        orientation 0 (RC) and (y, x) for orientation 1 (CR)
  sigma_t = sqrt(2 ln 2) / (pi * B * f0): Gaussian envelope whose -6 dB
        amplitude bandwidth is the fractional bandwidth B (65%, Section II-C)

The Gaussian is evaluated over every sample (no truncation).  Noise follows
the counter-based convention in oracle.philox.
"""
from __future__ import annotations

import numpy as np

from .philox import channel_noise


def pulse_sigma(cfg) -> float:
    return np.sqrt(2.0 * np.log(2.0)) / (np.pi * cfg.probe.bandwidth * cfg.probe.f0)


def delays(cfg, pos_f, o: int, k: int) -> np.ndarray:
    """Round-trip delays tau[S][Nc] for scatterer positions pos_f [S][3]."""
    pr = cfg.probe
    theta = cfg.seq.angles_rad[k]
    x, y, z = pos_f[:, 0], pos_f[:, 1], pos_f[:, 2]
    u, v = (x, y) if o == 0 else (y, x)
    L = (pr.n_elem - 1) * pr.pitch
    tau_tx = (z * np.cos(theta) + v * np.sin(theta) + 0.5 * L * abs(np.sin(theta))) / pr.c
    pe = (np.arange(pr.n_elem) - 0.5 * (pr.n_elem - 1)) * pr.pitch
    tau_rx = np.sqrt((u[:, None] - pe[None, :]) ** 2 + z[:, None] ** 2) / pr.c
    return tau_tx[:, None] + tau_rx


def simulate(cfg, medium, frames=None, with_noise: bool = True,
             scat_chunk: int = 64) -> np.ndarray:
    """IQ channel data [F][O][K][Nc][Ns] complex128 for the given frames."""
    F_all = cfg.seq.n_frames
    frames = list(range(F_all)) if frames is None else list(frames)
    K = cfg.n_angles
    Nc = cfg.probe.n_elem
    Ns = cfg.seq.n_samp
    t = cfg.seq.t_start + np.arange(Ns) / cfg.probe.fs
    sig = pulse_sigma(cfg)
    out = np.zeros((len(frames), 2, K, Nc, Ns), dtype=np.complex128)
    for fi, f in enumerate(frames):
        pos = medium.pos[f]
        for o in range(2):
            for k in range(K):
                tau = delays(cfg, pos, o, k)                        # [S][Nc]
                acc = np.zeros((Nc, Ns), dtype=np.complex128)
                for s0 in range(0, tau.shape[0], scat_chunk):
                    tt = tau[s0:s0 + scat_chunk]                    # [s][Nc]
                    a = medium.amp[s0:s0 + scat_chunk]
                    env = np.exp(-((t[None, None, :] - tt[:, :, None]) ** 2) / (2 * sig * sig))
                    ph = a[:, None] * np.exp(-2j * np.pi * cfg.probe.f0 * tt)   # [s][Nc]
                    acc += np.einsum("sc,sct->ct", ph, env)
                out[fi, o, k] = acc
        if with_noise and medium.noise_sigma > 0:
            block = 2 * K * Nc * Ns
            out[fi] += channel_noise(f * block, block, medium.noise_seed,
                                     medium.noise_sigma).reshape(2, K, Nc, Ns)
    return out
