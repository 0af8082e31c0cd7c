"""GPU parity of the XZ/YZ pairing (projection-based 3D localisation) against
the oracle, through the C ABI, on seeded plane localisation lists.

Pairing is index and selection work: the paired record indices, frames and the
copied coordinates must be identical, and the mean depth bit-identical (one
FP32 add and halving on both sides)."""
from dataclasses import replace

import numpy as np
import pytest

from synth import cfg_paper, cfg_tiny, plane_records, with_blocks, with_frames, with_angles
from oracle import pairing
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ulm():
    import paper_2511_21647_amd as u
    return u


def _ragged_cfg():
    c = with_blocks(with_angles(with_frames(cfg_tiny(), 18), [-6, -2, 0, 3, 6]), 4)
    g = c.grid
    return c.with_(grid=replace(g, nu=45, nz=37, u0=-22 * g.du, nv=45, v0=-22 * g.dv))


def _upload(torch, recs, capacity):
    rows = np.zeros((max(capacity, 1), 8), np.int32)
    raw = np.ascontiguousarray(recs).view(np.int32).reshape(-1, 8)
    rows[:len(raw)] = raw[:len(rows)]
    return torch.from_numpy(rows).cuda()


def _run(torch, ulm, cfg, recs, capacity=None, count=None, out_capacity=None):
    capacity = len(recs) if capacity is None else capacity
    count = len(recs) if count is None else count
    locs = _upload(torch, recs, capacity)
    cnt = torch.tensor([count], dtype=torch.int32, device="cuda")
    ctx = ulm.Context(cfg)
    out_capacity = 4 * max(len(recs), 1) if out_capacity is None else out_capacity
    out, oc = ulm.ulm_pair_planes(ctx, locs, cnt, capacity, out_capacity)
    torch.cuda.synchronize()
    return ctx, out, oc, int(oc.item())


def _check_equal(got, want):
    assert len(got) == len(want), (len(got), len(want))
    for f in ("frame", "idx_xz", "idx_yz", "x", "y", "z", "i_xz", "i_yz"):
        assert np.array_equal(got[f], want[f]), f


CASES = {
    # name: (cfg factory, mb per frame, seed, single-view fraction)
    "tiny": (cfg_tiny, 6, 11, 0.2),
    "tiny_dense": (cfg_tiny, 60, 12, 0.3),
    "ragged_b4": (_ragged_cfg, 8, 13, 0.2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_pairing_parity(torch, ulm, case):
    make, mb, seed, single = CASES[case]
    cfg = make()
    g = cfg.grid
    recs, _ = plane_records(g.nz, g.nv, g.n_blocks, cfg.seq.n_frames, mb, seed, single_frac=single)
    say(f"[pairing {case}] {len(recs)} records, B={g.n_blocks}, F={cfg.seq.n_frames}")
    want = pairing.pair_localisations(recs, g.n_blocks, g.nv)
    _, out, oc, n = _run(torch, ulm, cfg, recs)
    got = ulm.loc3d_to_numpy(out, oc)
    say(f"  pairs gpu {n} oracle {len(want)}")
    assert n == len(want) and len(want) > 0
    _check_equal(got, want)


@pytest.mark.parametrize("blocks", [1, 8])
def test_pairing_paper_scale(torch, ulm, blocks):
    """300 frames of 250 x 274 planes, ~40 MBs per frame (one slab, and the
    eight-slab split)."""
    cfg = with_blocks(cfg_paper(), blocks)
    g = cfg.grid
    recs, _ = plane_records(g.nz, g.nv, blocks, cfg.seq.n_frames, 40, 21 + blocks)
    say(f"[pairing paper B={blocks}] {len(recs)} records")
    want = pairing.pair_localisations(recs, blocks, g.nv)
    _, out, oc, n = _run(torch, ulm, cfg, recs)
    say(f"  pairs gpu {n} oracle {len(want)}")
    assert n == len(want) and len(want) > 1000
    _check_equal(ulm.loc3d_to_numpy(out, oc), want)


def test_pairing_edge_cases(torch, ulm):
    cfg = cfg_tiny()
    g = cfg.grid
    recs, _ = plane_records(g.nz, g.nv, 1, cfg.seq.n_frames, 6, 31)
    want = pairing.pair_localisations(recs, 1, g.nv)
    # empty list
    _, _, _, n = _run(torch, ulm, cfg, recs[:0], capacity=0, count=0, out_capacity=8)
    assert n == 0
    # localiser overflow: count beyond capacity, only the stored records are paired
    cap = len(recs) * 2 // 3
    _, out, oc, n = _run(torch, ulm, cfg, recs, capacity=cap, count=len(recs) + 50)
    w2 = pairing.pair_localisations(recs[:cap], 1, g.nv)
    _check_equal(ulm.loc3d_to_numpy(out, oc), w2)
    # output overflow: the total is reported, the first out_capacity pairs written
    oc_cap = len(want) // 2
    ctx, out, oc, n = _run(torch, ulm, cfg, recs, out_capacity=oc_cap)
    assert n == len(want)
    _check_equal(ulm.loc3d_to_numpy(out, oc), want[:oc_cap])
    with pytest.raises(ulm.ULMError) as e:
        ulm.ulm_check_status(ctx, oc, oc_cap)
    assert e.value.code == ulm.ULM_ERR_OVERFLOW
    # one orientation only: no pairs
    xz = recs[recs["plane"] == 0]
    _, _, _, n = _run(torch, ulm, cfg, xz)
    assert n == 0
