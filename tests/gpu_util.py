"""Helpers for the GPU parity tests (comparison rules, not method arithmetic)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def undecidable_mask(I, N, fmax, tau, alpha, delta):
    """Pixels whose detection decision lies within `delta` of a threshold or a
    neighbour comparison (for one image)."""
    nz, nu = N.shape
    near_ncc = np.abs(N - tau) <= delta
    near_int = (np.abs(I / max(fmax, 1e-300) - alpha) <= delta) & (N >= tau - delta)
    pad = np.full((nz + 2, nu + 2), -np.inf)
    pad[1:-1, 1:-1] = N
    gap = np.full((nz, nu), np.inf)
    for dz in (-1, 0, 1):
        for du in (-1, 0, 1):
            if dz == 0 and du == 0:
                continue
            q = pad[1 + dz:1 + dz + nz, 1 + du:1 + du + nu]
            gap = np.minimum(gap, np.abs(N - q))
    near_max = (gap <= delta) & (N >= tau - delta) & (I >= (alpha - delta) * fmax)
    return near_ncc | near_int | near_max


def compare_detections(gpu, ora, N, I, cfg, delta, pos_tol):
    """gpu: structured records from the library; ora: oracle records.
    N, I: oracle NCC maps / envelopes [O][B][F][nz][nu].
    Returns (n_matched, n_undecidable, max_position_error)."""
    O, B, F = N.shape[:3]
    und = set()
    for o in range(O):
        for b in range(B):
            for f in range(F):
                fm = float(I[o, b, f].max())
                m = undecidable_mask(I[o, b, f], N[o, b, f], fm, cfg.loc.tau_ncc, cfg.loc.alpha,
                                     delta)
                for z, u in zip(*np.nonzero(m)):
                    und.add((o * B + b, f, int(z), int(u)))
    g = {(int(r["plane"]), int(r["frame"]), int(r["iz"]), int(r["iu"])): r for r in gpu}
    oo = {(int(r["plane"]) * B + int(r["block"]), int(r["frame"]), int(r["iz"]), int(r["iu"])): r
          for r in ora}
    gd = set(g) - und
    od = set(oo) - und
    assert gd == od, (f"decidable sets differ: only GPU {sorted(gd - od)[:10]}, "
                      f"only oracle {sorted(od - gd)[:10]}")
    err = 0.0
    for key in gd:
        a, b = g[key], oo[key]
        err = max(err, abs(float(a["z"]) - float(b["z"])), abs(float(a["u"]) - float(b["u"])))
    assert err <= pos_tol, err
    # the GPU output order is (plane, frame, iz, iu)
    keys = [(int(r["plane"]), int(r["frame"]), int(r["iz"]), int(r["iu"])) for r in gpu]
    assert keys == sorted(keys)
    return len(gd), len((set(g) | set(oo)) & und), err
