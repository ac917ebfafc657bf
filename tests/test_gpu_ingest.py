"""Frame ingest on the GPU (letterbox + bilinear resize + /255, HWC uint8 ->
NCHW FP32) against the FP64 oracle, element by element."""

import sys

import numpy as np
import pytest

from jde_inputs import FULL, capture_frame
from oracle.ingest import ingest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("src_hw,targets", [
    ((1080, 1920), [(608, 1088), (320, 576)]),      # FullHD, as the paper's inputs; a ragged pair of targets
    ((480, 640), [(608, 1088)]),                     # 4:3 source: pillar-boxed
    ((97, 150), [(192, 320), (64, 96)]),             # upsampling and odd sizes
])
def test_ingest_matches_oracle(src_hw, targets):
    import torch
    from paper_2011_03910_amd import jde_ingest
    assert torch.cuda.is_available()
    H, W = src_hw
    n = len(targets)
    _say(f"case: ingest {W}x{H} -> {targets}")
    src = np.stack([capture_frame(FULL.seed, 7, t, H, W) for t in range(n)])
    out = jde_ingest(torch.from_numpy(src).cuda(), targets)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    off = 0
    for f, (h, w) in enumerate(targets):
        ref = ingest(src[f], h, w)
        g = got[off:off + 3 * h * w].reshape(3, h, w)
        off += 3 * h * w
        err = float(np.abs(g - ref).max())
        _say(f"  frame {f} {w}x{h}: max abs err {err:.2e}")
        assert err <= 1e-6
    assert off == got.size
