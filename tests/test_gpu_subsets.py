"""The paper's order after the clutter filter, on the tiny ensemble: MB
separation into up/down x speed subsets, NCC localisation of every subset and
XZ/YZ pairing of every subset's detections, all through the C ABI.

Each step is compared with the oracle on the library's own input to that step
(the filtered planes, the subsets, the detection lists), so a difference is
attributed to the step that made it."""
import numpy as np
import pytest

from synth import cfg_tiny
from oracle import localize, pairing, separation
from gpu_util import compare_detections, rel_l2, say

pytestmark = pytest.mark.gpu

S = 2


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def ulm():
    import paper_2511_21647_amd as u
    return u


def test_subset_pipeline_tiny(torch, ulm, tiny_iq):
    cfg = cfg_tiny()
    ctx = ulm.Context(cfg)
    iq = torch.from_numpy(np.ascontiguousarray(tiny_iq.astype(np.complex64))).cuda()
    proj = ulm.rca_beamform_proj(ctx, iq)
    ulm.svd_clutter_filter(ctx, proj)
    ulm.ulm_check_status(ctx)
    sub = ulm.ulm_separate(ctx, proj, S)
    torch.cuda.synchronize()
    ref = separation.separate(proj.cpu().numpy().astype(np.complex128), S)
    got_sub = sub.cpu().numpy()
    e = max(rel_l2(got_sub[i], ref[i]) for i in range(2 * S))
    say(f"[subsets tiny] separation worst rel-L2 {e:.2e}")
    assert e <= 1e-5
    cap = 100000
    total_pairs = 0
    for i in range(2 * S):
        locs, cnt = ulm.ncc_localize(ctx, sub[i].contiguous(), cap)
        ulm.ulm_check_status(ctx, cnt, cap)
        got = ulm.locs_to_numpy(locs, cnt)
        ora, N, I = localize.localize(got_sub[i].astype(np.complex128), cfg)
        n, nund, err = compare_detections(got, ora, N, I, cfg, delta=1e-4, pos_tol=1e-3)
        out, oc = ulm.ulm_pair_planes(ctx, locs, cnt, cap, 4 * cap)
        ulm.ulm_check_status(ctx, oc, 4 * cap)
        pairs = ulm.loc3d_to_numpy(out, oc)
        want = pairing.pair_localisations(got, cfg.grid.n_blocks, cfg.grid.nv)
        say(f"  subset {i}: {len(got)} detections (matched {n}, undecidable {nund}, "
            f"max pos err {err:.1e}), {len(pairs)} 3D pairs")
        assert len(pairs) == len(want)
        for f in ("frame", "idx_xz", "idx_yz", "x", "y", "z"):
            assert np.array_equal(pairs[f], want[f]), f
        total_pairs += len(pairs)
    assert total_pairs > 0
