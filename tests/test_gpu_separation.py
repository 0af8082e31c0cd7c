"""GPU parity of the MB separation (temporal DFT, up/down x speed-range masks,
inverse DFT) against the oracle, through the C ABI, on seeded planes: tiny and
ragged sizes in full, and the paper-scale 300-frame planes on sampled pixels
plus the partition property over every pixel."""
from dataclasses import replace

import numpy as np
import pytest

from synth import arrays, cfg_paper, cfg_tiny, with_angles, with_blocks, with_frames
from oracle import separation
from gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu

TOL = 1e-5          # relative L2 per subset (FP32 transforms of length <= 300)


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


@pytest.mark.parametrize("case,S", [("tiny", 3), ("tiny", 1), ("ragged", 2), ("ragged", 8)])
def test_separation_parity(torch, ulm, case, S):
    cfg = cfg_tiny() if case == "tiny" else _ragged_cfg()
    ctx = ulm.Context(cfg)
    x = arrays.complex_normal(ctx.proj_shape, seed=61 + S)
    say(f"[separation {case} S={S}] planes {x.shape}")
    sub = ulm.ulm_separate(ctx, torch.from_numpy(x).cuda(), S)
    torch.cuda.synchronize()
    got = sub.cpu().numpy()
    ref = separation.separate(x.astype(np.complex128), S)
    errs = [rel_l2(got[i], ref[i]) for i in range(2 * S) if np.linalg.norm(ref[i]) > 0]
    say(f"  worst subset rel-L2 {max(errs):.2e}")
    assert max(errs) <= TOL
    for i in range(2 * S):
        if np.linalg.norm(ref[i]) == 0:            # an empty speed range gives zeros
            assert np.all(got[i] == 0)


def test_separation_paper_scale(torch, ulm):
    cfg = cfg_paper()
    g = cfg.grid
    F, S = cfg.seq.n_frames, 3
    ctx = ulm.Context(cfg)
    x = arrays.complex_normal(ctx.proj_shape, seed=71)
    d = torch.from_numpy(x).cuda()
    sub = ulm.ulm_separate(ctx, d, S)
    torch.cuda.synchronize()
    # sampled pixels of both planes against the oracle
    rng = np.random.default_rng(72)
    pix = np.sort(rng.choice(g.nz * g.nu, 3000, replace=False))
    flat = x.reshape(2, 1, F, g.nz * g.nu)[:, :, :, pix]
    ref = separation.separate(flat[..., None].astype(np.complex128), S)[..., 0]
    got = sub.reshape(2 * S, 2, 1, F, g.nz * g.nu)[..., torch.from_numpy(pix).cuda()].cpu().numpy()
    errs = [rel_l2(got[i], ref[i]) for i in range(2 * S)]
    say(f"[separation paper] {len(pix)} sampled pixels, worst subset rel-L2 {max(errs):.2e}")
    assert max(errs) <= TOL
    # every pixel: the subsets plus the DC and Nyquist components give the planes back
    total = sub.sum(dim=0)
    X = torch.fft.fft(d.to(torch.complex128), dim=2)
    keep = torch.zeros_like(X)
    keep[:, :, 0] = X[:, :, 0]
    keep[:, :, F // 2] = X[:, :, F // 2]
    rest = torch.fft.ifft(keep, dim=2)
    e = (torch.linalg.vector_norm(total.to(torch.complex128) + rest - d.to(torch.complex128)) /
         torch.linalg.vector_norm(d.to(torch.complex128))).item()
    say(f"  partition over every pixel: rel-L2 {e:.2e}")
    assert e <= TOL


def test_separation_argument_checks(torch, ulm):
    ctx = ulm.Context(cfg_tiny())
    x = torch.zeros(ctx.proj_shape, dtype=torch.complex64, device="cuda")
    for S in (0, 9):
        with pytest.raises(ulm.ULMError) as e:
            ulm.ulm_separate(ctx, x, S)
        assert e.value.code == ulm.ULM_ERR_INVALID_ARG
    ctx37 = ulm.Context(with_frames(cfg_tiny(), 37))      # prime frame count above 7
    x37 = torch.zeros(ctx37.proj_shape, dtype=torch.complex64, device="cuda")
    with pytest.raises(ulm.ULMError) as e:
        ulm.ulm_separate(ctx37, x37, 3)
    assert e.value.code == ulm.ULM_ERR_INVALID_ARG
