"""Pins of the XZ/YZ pairing oracle (CPU only)."""
import numpy as np

from oracle import pairing


def _recs(rows):
    """rows: (plane, frame, z, u, intensity)."""
    a = np.zeros(len(rows), dtype=[("plane", "i4"), ("frame", "i4"), ("z", "f4"), ("u", "f4"),
                                   ("intensity", "f4")])
    for k, r in enumerate(rows):
        a[k] = r
    return a


def test_recovers_separated_points_exactly():
    """Well separated 3D points (distinct depths, equal intensities in both
    projections) come back with x from XZ, y from YZ and z as the mean."""
    rng = np.random.default_rng(0)
    pts = []
    for k in range(12):
        pts.append((rng.uniform(0, 200), rng.uniform(0, 200), 10.0 + 7.0 * k, rng.uniform(1, 5)))
    rows = []
    for (x, y, z, I) in pts:
        rows.append((0, 3, z + 0.2, x, I))
        rows.append((1, 3, z - 0.1, y, I))
    out = pairing.pair_localisations(_recs(rows), 1, 274)
    assert len(out) == len(pts)
    got = sorted((round(float(r["x"]), 4), round(float(r["y"]), 4), round(float(r["z"]), 4)) for r in out)
    want = sorted((round(float(np.float32(x)), 4), round(float(np.float32(y)), 4),
                   round(float((np.float32(z + 0.2) + np.float32(z - 0.1)) * np.float32(0.5)), 4))
                  for (x, y, z, I) in pts)
    assert got == want


def test_ratio_gate_and_axial_tolerance():
    base = [(0, 0, 50.0, 10.0, 1.0)]
    # ratio 1.2 and 0.85: rejected; 1.1 accepted
    for ratio, paired in ((1.2, False), (0.85, False), (1.1, True), (0.91, True)):
        out = pairing.pair_localisations(_recs(base + [(1, 0, 50.0, 20.0, 1.0 / ratio)]), 1, 274)
        assert (len(out) == 1) == paired, ratio
    # one voxel axially: accepted; beyond: rejected
    for dz, paired in ((1.0, True), (1.02, False), (-0.99, True)):
        out = pairing.pair_localisations(_recs(base + [(1, 0, 50.0 + dz, 20.0, 1.0)]), 1, 274)
        assert (len(out) == 1) == paired, dz


def test_mutual_minimum_resolves_conflicts():
    """Two XZ records compete for one YZ record: the closer ratio wins and the
    other stays unpaired even though its own best candidate is that record."""
    rows = [(0, 0, 40.0, 5.0, 1.00), (0, 0, 40.5, 9.0, 1.04), (1, 0, 40.2, 7.0, 1.00)]
    out = pairing.pair_localisations(_recs(rows), 1, 274)
    assert len(out) == 1 and int(out[0]["idx_xz"]) == 0 and int(out[0]["idx_yz"]) == 2
    # frames never mix
    rows2 = rows + [(1, 1, 40.5, 3.0, 1.04)]
    out2 = pairing.pair_localisations(_recs(rows2), 1, 274)
    assert len(out2) == 1


def test_pairs_are_mutual_best_and_complete():
    """Random dense lists: every output pair is the mutual best by the stated
    closeness (checked with plain loops), and no mutually-best pair is missing."""
    rng = np.random.default_rng(5)
    rows = []
    for o in range(2):
        for _ in range(60):
            rows.append((o, 0, rng.uniform(0, 30), rng.uniform(0, 100), rng.uniform(0.5, 1.5)))
    recs = _recs(rows)
    out = pairing.pair_localisations(recs, 1, 274)
    A = [k for k in range(len(recs)) if recs["plane"][k] == 0]
    B = [k for k in range(len(recs)) if recs["plane"][k] == 1]

    def cost(a, b):
        Ia, Ib = np.float32(recs["intensity"][a]), np.float32(recs["intensity"][b])
        rho = np.float32(Ia / Ib)
        if abs(np.float32(recs["z"][a]) - np.float32(recs["z"][b])) > 1.0:
            return np.inf
        if not (np.float32(0.9) <= rho <= np.float32(1.11)):
            return np.inf
        return max(float(rho), float(np.float32(Ib / Ia)))

    best_b = {}
    for a in A:
        c = [(cost(a, b), b) for b in B]
        m = min(c)
        if np.isfinite(m[0]):
            best_b[a] = min(b for (v, b) in c if v == m[0])
    best_a = {}
    for b in B:
        c = [(cost(a, b), a) for a in A]
        m = min(c)
        if np.isfinite(m[0]):
            best_a[b] = min(a for (v, a) in c if v == m[0])
    want = sorted((a, b) for a, b in best_b.items() if best_a.get(b) == a)
    got = sorted((int(r["idx_xz"]), int(r["idx_yz"])) for r in out)
    assert got == want and len(got) > 5


def test_swap_symmetry():
    """Exchanging the roles of the two planes (x <-> y) gives the same pairs."""
    rng = np.random.default_rng(9)
    rows = [(o, 2, rng.uniform(0, 20), rng.uniform(0, 50), rng.uniform(0.8, 1.2))
            for o in range(2) for _ in range(25)]
    recs = _recs(rows)
    swapped = recs.copy()
    swapped["plane"] = 1 - recs["plane"]
    a = pairing.pair_localisations(recs, 1, 274)
    b = pairing.pair_localisations(swapped, 1, 274)
    assert sorted(zip(a["idx_xz"], a["idx_yz"])) == sorted(zip(b["idx_yz"], b["idx_xz"]))
    assert np.allclose(sorted(a["z"]), sorted(b["z"]))


def test_slab_consistency():
    """With two slabs (width 137 of 274 pixels), an XZ record of slab b pairs
    only with a YZ record whose y lies in slab b and whose own slab holds the
    XZ record's x."""
    # XZ slab 0 (y < 137) at x = 200 (slab 1); YZ slab 1 at y = 100 (slab 0): consistent
    good = [(0, 0, 30.0, 200.0, 1.0), (3, 0, 30.2, 100.0, 1.0)]
    assert len(pairing.pair_localisations(_recs(good), 2, 274)) == 1
    # y of the YZ record in the other slab
    bad_y = [(0, 0, 30.0, 200.0, 1.0), (3, 0, 30.2, 150.0, 1.0)]
    assert len(pairing.pair_localisations(_recs(bad_y), 2, 274)) == 0
    # x of the XZ record outside the YZ record's slab
    bad_x = [(0, 0, 30.0, 20.0, 1.0), (3, 0, 30.2, 100.0, 1.0)]
    assert len(pairing.pair_localisations(_recs(bad_x), 2, 274)) == 0
    # the boundary pixel: y = 136.49 rounds to pixel 136 (slab 0), 136.5 to 137 (slab 1)
    edge = [(0, 0, 30.0, 200.0, 1.0), (3, 0, 30.2, 136.49, 1.0)]
    assert len(pairing.pair_localisations(_recs(edge), 2, 274)) == 1
    edge[1] = (3, 0, 30.2, 136.5, 1.0)
    assert len(pairing.pair_localisations(_recs(edge), 2, 274)) == 0


def test_synthetic_lists_recover_most_points():
    """On the seeded plane lists used by the GPU tests, sparse MBs seen by both
    planes come back: recovered 3D positions lie within 1.5 px of a true MB,
    and most MBs are found."""
    from synth import plane_records
    recs, truth = plane_records(64, 64, 1, 3, 4, seed=3, single_frac=0.0)
    out = pairing.pair_localisations(recs, 1, 64)
    found = 0
    for f in range(3):
        t = truth[f]
        got = out[out["frame"] == f]
        for r in got:
            d = np.sqrt((t[:, 0] - r["x"]) ** 2 + (t[:, 1] - r["y"]) ** 2 + (t[:, 2] - r["z"]) ** 2)
            assert d.min() < 1.5
        found += len(got)
    n = sum(len(t) for t in truth)
    assert found >= 0.7 * n, (found, n)


def test_chunked_cost_matrix_gives_the_same_pairs():
    """Forming the cost matrix a few rows at a time changes nothing, ties
    included (equal intensities everywhere make every candidate cost 1)."""
    rng = np.random.default_rng(0)
    dt = [("z", "f4"), ("u", "f4"), ("intensity", "f4"), ("block", "i8")]
    for equal in (False, True):
        xz, yz = np.zeros(300, dt), np.zeros(280, dt)
        for a in (xz, yz):
            a["z"] = rng.uniform(0, 5, len(a))
            a["u"] = rng.uniform(0, 64, len(a))
            a["intensity"] = 1.0 if equal else rng.uniform(0.9, 1.1, len(a))
            a["block"] = rng.integers(0, 4, len(a))
        for per in (None, 16):
            whole = pairing.pair_frame(xz, yz, per, chunk=100000)
            assert pairing.pair_frame(xz, yz, per, chunk=7) == whole and len(whole) >= 3
