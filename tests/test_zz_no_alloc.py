"""The allocation-free pairing entry point (library-owned scratch array) against
the workspace entry point, through the C ABI: identical pairs on two calls in a
row, the second with a smaller input, on the tiny geometry and on a ragged
four-slab geometry; capacities beyond the array are refused before any launch."""
from dataclasses import replace

import numpy as np
import pytest

from synth import cfg_tiny, plane_records, with_angles, with_blocks, with_frames
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


@pytest.mark.parametrize("case", ["tiny", "ragged_b4"])
def test_noalloc_pairing_matches_workspace_entry(torch, ulm, case):
    cfg = cfg_tiny() if case == "tiny" else _ragged_cfg()
    g = cfg.grid
    ctx = ulm.Context(cfg)
    # two calls in a row on the same device array, the second input smaller
    for call, (mb, seed) in enumerate(((60, 21), (7, 22))):
        recs, _ = plane_records(g.nz, g.nv, g.n_blocks, cfg.seq.n_frames, mb, seed,
                                single_frac=0.25)
        cap = len(recs)
        out_cap = 4 * max(cap, 1)
        say(f"[noalloc {case} call {call}] {cap} records, B={g.n_blocks}")
        locs = _upload(torch, recs, cap)
        cnt = torch.tensor([cap], dtype=torch.int32, device="cuda")
        want, want_n = ulm.ulm_pair_planes(ctx, locs, cnt, cap, out_cap)
        out = torch.full((out_cap, 8), -7, dtype=torch.int32, device="cuda")
        out_n = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        ulm.ulm_pair_planes_noalloc(ctx, locs, cnt, cap, out_cap, out, out_n)
        torch.cuda.synchronize()
        n = int(want_n.item())
        assert n > 0
        assert int(out_n.item()) == n
        assert torch.equal(out[:n], want[:n])
        say(f"  {n} pairs, identical")
    ctx.close()


def test_noalloc_pairing_refuses_capacity_beyond_scratch(torch, ulm):
    cfg = cfg_tiny()
    ctx = ulm.Context(cfg)
    cap = ulm.ULM_NOALLOC_SCRATCH_BYTES // 4          # 4 bytes per record in the workspace
    locs = torch.zeros((cap, 8), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.zeros((1, 8), dtype=torch.int32, device="cuda")
    out_n = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(ulm.ULMError) as ei:
        ulm.ulm_pair_planes_noalloc(ctx, locs, cnt, cap, 1, out, out_n)
    assert ei.value.code == ulm.ULM_ERR_INVALID_ARG
    assert "scratch" in str(ei.value)
    ctx.close()
