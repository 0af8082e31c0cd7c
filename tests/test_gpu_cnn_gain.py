"""What the trained network gains over the method without it.

One held-out paper-scale ensemble (seed disjoint from every training ensemble,
6000 MBs on vessel splines) is simulated, beamformed and clutter-filtered by
the library; the NCC localiser and the trained CNN then localise the same
filtered planes.  Against the true MB positions (one-to-one matching within
0.5 px per image), the CNN must find more MBs than NCC at a higher precision
and with a smaller position error."""
import os

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

HELDOUT = 19999     # not a training (0, 1, ...) or evaluation (10000, 10001, ...) ensemble
N_MB = 6000


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def test_cnn_gains_over_ncc(torch):
    import paper_2511_21647_amd as ulm
    from paper_2511_21647_amd import train_cnn as tc
    from synth import cfg_cnn, make_medium, plane_positions

    cfg = cfg_cnn(N_MB)
    F = cfg.seq.n_frames
    med = make_medium(cfg, HELDOUT)
    ctx = ulm.Context(cfg, precision=ulm.ULM_PREC_BF16X3)
    iq = ulm.ulm_sim_channel_data(ctx, torch.from_numpy(med.pos).cuda(),
                                  torch.from_numpy(med.amp).cuda(), med.noise_seed,
                                  med.noise_sigma)
    proj = ulm.rca_beamform_proj(ctx, iq)
    del iq
    ulm.svd_clutter_filter(ctx, proj)
    ulm.ulm_check_status(ctx)
    labels = plane_positions(cfg, med)
    truth = [labels[n // F][n % F] for n in range(2 * F)]
    cap = 4_000_000
    locs, cnt = ulm.ncc_localize(ctx, proj, cap)
    ulm.ulm_check_status(ctx, cnt, cap)
    ncc = tc.per_image(ulm.locs_to_numpy(locs, cnt), 2 * F, F)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    w = np.load(os.path.join(root, "paper_2511_21647_amd", "weights", "cnn_paper.npy"))
    params = torch.from_numpy(w.astype(np.float32)).cuda()
    locs, cnt = ulm.ulm_cnn_localize(ctx, params, proj, cap, ulm.CNN_THRESHOLD, 64, ulm.ULM_CNN_BF16,
                                     locs, cnt)
    ulm.ulm_check_status(ctx, cnt, cap)
    cnn = tc.per_image(ulm.locs_to_numpy(locs, cnt), 2 * F, F)
    s_ncc, s_cnn = tc.score(ncc, truth), tc.score(cnn, truth)
    s_agree = tc.score(cnn, ncc)
    say(f"[cnn gain] NCC vs truth: {s_ncc}")
    say(f"[cnn gain] CNN vs truth: {s_cnn}")
    say(f"[cnn gain] CNN vs NCC:   {s_agree}")
    assert s_cnn["recall"] > s_ncc["recall"]
    assert s_cnn["precision"] > s_ncc["precision"]
    assert s_cnn["rms_px"] < s_ncc["rms_px"]
