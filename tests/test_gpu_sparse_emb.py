"""Deferred sparse embedding head: the emb 3x3 conv run at kept cells only,
after NMS, against the dense emb map at the same cells (same network, same
detections) and against the FP64 oracle's normalised embeddings."""

import sys

import numpy as np
import pytest

from jde_inputs import TINY, FULL
from oracle import post as opost
from tests.helpers import weights, frames, oracle_forward, gpu_dets, anchors, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible MI355X"
    return t


def _run(torch, cfg, precision, k, n, descs, sparse, cap=512, conf=0.5, fr=None):
    from paper_2011_03910_amd import JDE
    m = JDE(cfg.c0, cfg.blocks, cfg.emb_dim, anchors(cfg.name), precision, n, cfg.height, cfg.width, cap)
    m.load_weights(weights(cfg.name, k))
    m.sparse_emb(sparse)
    x = torch.from_numpy(np.ascontiguousarray(fr)).cuda().reshape(-1)
    heads = m.forward(x, descs, heads=m.head_buffers(descs, emb=not sparse))
    d = m.decode(heads, descs, conf_thr=conf)
    torch.cuda.synchronize()
    return m, d


@pytest.mark.parametrize("cfg_name,precision,k,n,conf", [
    ("tiny", "fp32", 50, 3, 0.5),
    ("tiny", "bf16", 50, 2, 0.3),
    pytest.param("full", "fp32", 1000, 1, 0.5, marks=pytest.mark.slow),
    pytest.param("full", "bf16", 40, 4, 0.5, marks=pytest.mark.slow),
    pytest.param("full", "fp16", 100, 2, 0.5, marks=pytest.mark.slow),
])
def test_sparse_emb_equals_dense_emb_at_kept_cells(torch, cfg_name, precision, k, n, conf):
    cfg = TINY if cfg_name == "tiny" else FULL
    _say(f"case: sparse emb {cfg_name} {precision} K={k} n={n} conf={conf}")
    descs = [(cfg.height, cfg.width)] * n
    fr = frames(cfg_name, n)
    md, dd = _run(torch, cfg, precision, k, n, descs, False, conf=conf, fr=fr)
    ms, ds = _run(torch, cfg, precision, k, n, descs, True, conf=conf, fr=fr)
    worst = 0.0
    total = 0
    for f in range(n):
        a, b = gpu_dets(dd, f, md.cap), gpu_dets(ds, f, ms.cap)
        # identical detections (the det branch is the same launch either way)
        for key in ("anchor_idx", "margins", "boxes", "scores"):
            np.testing.assert_array_equal(a[key], b[key])
        if len(a["emb"]):
            worst = max(worst, float(np.abs(a["emb"] - b["emb"]).max()))
            np.testing.assert_allclose(np.linalg.norm(b["emb"], axis=1), 1.0, atol=1e-6)
        total += len(a["emb"])
    _say(f"  {total} detections; max |sparse - dense| of the unit embeddings {worst:.2e}")
    assert total > 0 and worst == 0.0    # same MFMA sequence as the dense conv: bitwise equal


def test_sparse_emb_tiny_fp32_vs_oracle(torch):
    """FP32 sparse embeddings of the kept detections against the oracle's
    normalised FP64 embeddings (same detections)."""
    _say("case: sparse emb tiny fp32 vs oracle")
    ms, ds = _run(torch, TINY, "fp32", 50, 1, [(192, 320)], True, fr=frames("tiny", 1))
    g = gpu_dets(ds, 0, ms.cap)
    r = opost.detections(oracle_forward("tiny", 50, 1), anchors("tiny"), 0.5, 0.4)
    np.testing.assert_array_equal(g["anchor_idx"], r["idx"])
    e = rel_err(g["emb"], r["emb"])
    _say(f"  {len(g['emb'])} detections, emb rel err vs fp64 {e:.2e}")
    assert e <= 1e-4
