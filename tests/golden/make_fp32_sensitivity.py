"""Writes fp32_sensitivity_tiny.json: how much the oracle's own clutter filter
and localiser move when their input projections carry FP32-sized errors.

The plain GPU path stores its projections in FP32, and the clutter filter
amplifies their relative error by the tissue-to-residual ratio.  The whole-path
comparison of the GPU with the oracle (IQ -> detections) therefore cannot be
tighter than the oracle's own response to such an input error.  This script
measures that response on the tiny ensemble (ensemble 0, oracle-simulated
channel data) by running the oracle's filter and localiser on
  fp32            the FP64 projections rounded to complex64, and
  fp32_perturbed  the FP64 projections times (1 + eps z), z unit-rms complex
                  Gaussian (seeded), eps = 1e-6 (the random-walk size of FP32
                  summation over 32 elements x 4 transmits, sqrt(128) 2^-24,
                  rounded up), then rounded to complex64,
and comparing with the run on the FP64 projections.  It calls only oracle/ and
synth/.  Run from the repository root:  python tests/golden/make_fp32_sensitivity.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "fp32_sensitivity_tiny.json")
EPS = 1e-6
MARGIN = 1e-5            # a reference detection counts when all its margins exceed this
MB_SCALE = 0.2           # MB-scale peaks: envelope >= 0.2 x frame maximum


def _chain(P, cfg):
    from oracle import clutter, localize
    filt, _ = clutter.filter_planes(np.asarray(P, dtype=np.complex128), cfg.svd_cutoff)
    recs, N, I = localize.localize(filt, cfg)
    return filt, recs, N, I


def measure():
    from synth import arrays, cfg_tiny, make_medium
    from oracle import beamform, sim

    cfg = cfg_tiny()
    iq = sim.simulate(cfg, make_medium(cfg, 0))
    P = beamform.beamform_proj(iq, cfg)
    f0, r0, N0, I0 = _chain(P, cfg)
    key = lambda r: (int(r["plane"]), int(r["block"]), int(r["frame"]), int(r["iz"]), int(r["iu"]))
    ref = {key(r): r for r in r0 if r["margin"] > MARGIN}
    fmax = {k: float(I0[k[0], k[1], k[2]].max()) for k in ref}
    z = arrays.complex_normal(P.shape, seed=91, dtype=np.complex128)
    variants = {"fp32": P.astype(np.complex64),
                "fp32_perturbed": (P * (1.0 + EPS * z)).astype(np.complex64)}
    out = {"eps_perturb": EPS, "margin": MARGIN, "reference_detections": len(ref), "variants": {}}
    for name, Pv in variants.items():
        f1, r1, N1, I1 = _chain(Pv, cfg)
        got = {key(r): r for r in r1}
        missing = [k for k in ref if k not in got]
        dpos = [max(abs(got[k]["z"] - ref[k]["z"]), abs(got[k]["u"] - ref[k]["u"]))
                for k in ref if k in got]
        dpos_mb = [d for k, d in zip([k for k in ref if k in got], dpos)
                   if ref[k]["intensity"] >= MB_SCALE * fmax[k]]
        rel_int = np.abs(I1 - I0) / np.maximum(I0.max(axis=(3, 4), keepdims=True), 1e-300)
        out["variants"][name] = {
            "filtered_rel_l2": float(np.linalg.norm(f1 - f0) / np.linalg.norm(f0)),
            "max_abs_dncc": float(np.max(np.abs(N1 - N0))),
            "max_rel_dintensity": float(rel_int.max()),
            "max_dpos_decidable_px": float(max(dpos, default=0.0)),
            "max_dpos_mb_scale_px": float(max(dpos_mb, default=0.0)),
            "mb_scale_detections": len(dpos_mb),
            "missing_decidable": len(missing),
        }
    return out


def main():
    res = measure()
    with open(OUT, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
