"""One captured graph for any batch within the capacity: the same graph is
replayed for mixes of different frame counts and sizes, and each replay must
equal the eager forward + decode of that batch bitwise (same launches, same
tiles), with the frame table and batch header written before each replay."""

import json
import os
import sys

import numpy as np
import pytest

from jde_inputs import FULL, ragged_mix, mix_frames
from tests.helpers import weights, anchors, gpu_dets

pytestmark = pytest.mark.gpu

MIXES = [
    [(608, 1088)],
    [(320, 576), (480, 864), (320, 576), (320, 576)],
    [(480, 864), (608, 1088), (320, 576)],
    [(608, 1088)],
]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _tiles():
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2011_03910_amd",
                        "tiles_mi355x.json")
    return np.array(json.load(open(path))["bf16_b16"], dtype=np.int32)


@pytest.mark.parametrize("precision,sparse", [("bf16", True), ("fp16", False)])
def test_one_graph_serves_every_mix(precision, sparse):
    import torch
    from paper_2011_03910_amd import JDE
    assert torch.cuda.is_available()
    _say(f"case: graph for any batch, {precision}, sparse emb {sparse}")
    cap_pix = 2 * 608 * 1088
    m = JDE(FULL.c0, FULL.blocks, FULL.emb_dim, anchors("full"), precision, 6, 608, 1088, 512,
            max_pixels=cap_pix)
    m.load_weights(weights("full", 100))
    m.set_tiles(_tiles())
    m.sparse_emb(sparse)
    cap_descs = [(608, 1088)] * 2                 # the capacity in pixels
    heads = m.head_buffers(cap_descs, emb=not sparse)
    dets = m.dets_buffers(6)
    frames = torch.zeros(3 * cap_pix, dtype=torch.float32, device="cuda")
    off = torch.tensor([0.0, 0.5, -0.5, 1.0, 0.25, -1.0], dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    g = m.graph_capture_any(frames, heads, dets, stream=s, logit_offset=off)
    torch.cuda.synchronize()
    for k, descs in enumerate(MIXES):
        n = len(descs)
        fr = torch.from_numpy(mix_frames(FULL.seed, descs, stream_base=300 + k)).cuda()
        frames[:fr.numel()].copy_(fr)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.launch_batch(descs, stream=s)
        s.synchronize()
        got_h = {key: [None if t is None else t.clone() for t in heads[key]] for key in heads}
        got_d = {key: v.clone() for key, v in dets.items()}
        # the same batch, eager
        h2 = m.head_buffers(descs, emb=not sparse)
        m.forward(frames[:fr.numel()], descs, heads=h2)
        d2 = m.decode(h2, descs, logit_offset=off)
        torch.cuda.synchronize()
        for sc in range(3):
            a = got_h["det"][sc][:h2["det"][sc].numel()]
            assert torch.equal(a, h2["det"][sc]), (k, sc)
            if not sparse:
                assert torch.equal(got_h["emb"][sc][:h2["emb"][sc].numel()], h2["emb"][sc]), (k, sc)
        total = 0
        for f in range(n):
            x, y = gpu_dets(got_d, f, m.cap), gpu_dets(d2, f, m.cap)
            for key in ("anchor_idx", "margins", "boxes", "scores", "emb"):
                np.testing.assert_array_equal(x[key], y[key])
            assert x["n_cand"] == y["n_cand"]
            total += len(x["anchor_idx"])
        for f in range(n, 6):
            assert int(got_d["count"][f]) == 0 and int(got_d["n_cand"][f]) == 0
        _say(f"  mix {k}: {n} frames {sorted(set(descs))}: replay == eager, {total} detections")
