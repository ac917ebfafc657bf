"""Pins of the oracle's decode, threshold, sort, NMS and normalisation (CPU only)."""

import json
import math
import os

import numpy as np
import pytest

from jde_inputs import TINY, model_weights, tiny_frame, anchors_px
from oracle import network as net
from oracle import post

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _maps(shapes, fill=0.0):
    return [np.full(s, fill) for s in shapes]


def test_decode_zero_deltas_give_anchor_at_cell_centre():
    anchors = np.array([[[10, 30], [20, 60]], [[40, 120], [50, 150]], [[70, 210], [80, 240]]],
                       dtype=np.float32)
    maps = _maps([(4, 6, 12), (2, 3, 12), (1, 2, 12)])
    maps[1][1, 2, 6 + 5] = 1.0                      # scale 16, cell (1, 2), anchor 1: c_fg > c_bg
    c = post.decode_frame(maps, anchors, 0.5)
    # every anchor with c_fg == c_bg has score exactly 0.5 and is kept at thr 0.5
    assert len(c["idx"]) == (4 * 6 + 2 * 3 + 1 * 2) * 2
    sel = c["idx"] == 4 * 6 * 2 + 2 * (1 * 3 + 2) + 1
    assert sel.sum() == 1
    cx, cy = (2 + 0.5) * 16, (1 + 0.5) * 16
    np.testing.assert_array_equal(c["boxes"][sel][0], [cx - 25, cy - 75, cx + 25, cy + 75])
    assert c["score"][sel][0] == pytest.approx(1 / (1 + math.exp(-1.0)), rel=1e-15)
    assert np.all(c["score"][~sel] == 0.5)
    assert np.all(np.diff(c["idx"]) > 0)


def test_decode_delta_closed_forms():
    anchors = np.array([[[8, 24]], [[16, 48]], [[32, 96]]], dtype=np.float32)
    maps = _maps([(2, 2, 6), (1, 1, 6), (1, 1, 6)], fill=-1.0)
    for m in maps:
        m[..., 4] = 1.0                              # c_bg above c_fg: dropped
    maps[0][..., 4] = -1.0
    maps[0][..., 5] = 5.0                            # keep every stride-8 anchor
    maps[0][0, 0, :4] = [0.5, -0.25, math.log(2.0), 0.0]
    maps[0][0, 1, :4] = [0.0, 0.0, 10.0, -10.0]      # dw clipped at ln 64
    c = post.decode_frame(maps, anchors, 0.5)
    assert list(c["idx"]) == [0, 1, 2, 3]
    b0 = c["boxes"][0]
    np.testing.assert_allclose([(b0[0] + b0[2]) / 2, (b0[1] + b0[3]) / 2], [4 + 4, 4 - 6])
    np.testing.assert_allclose([b0[2] - b0[0], b0[3] - b0[1]], [16.0, 24.0])
    b1 = c["boxes"][1]
    np.testing.assert_allclose(b1[2] - b1[0], 8 * 64.0)
    np.testing.assert_allclose(b1[3] - b1[1], 24 * math.exp(-10.0))
    np.testing.assert_allclose(c["score"], 1 / (1 + math.exp(-6.0)))


def test_threshold_margin_test_equals_score_test(rng):
    for thr in (0.3, 0.5, 0.7, 0.9):
        m = rng.normal(0, 3, 20000)
        score = 1 / (1 + np.exp(-m))
        far = np.abs(score - thr) > 1e-9
        keep = m >= post.logit_threshold(thr)
        np.testing.assert_array_equal(keep[far], (score >= thr)[far])


def test_threshold_edges():
    maps = _maps([(1, 1, 6), (1, 1, 6), (1, 1, 6)])
    anchors = np.ones((3, 1, 2), dtype=np.float32)
    assert len(post.decode_frame(maps, anchors, 0.0)["idx"]) == 3
    assert len(post.decode_frame(maps, anchors, 1.0)["idx"]) == 0
    maps[0][0, 0, 5] = np.nan                         # NaN is never >= thr
    assert len(post.decode_frame(maps, anchors, 0.5)["idx"]) == 2


def _iou64(a, b):
    iw = max(0.0, min(a[2], b[2]) - max(a[0], b[0]))
    ih = max(0.0, min(a[3], b[3]) - max(a[1], b[1]))
    inter = iw * ih
    return inter / ((a[2] - a[0]) * (a[3] - a[1]) + (b[2] - b[0]) * (b[3] - b[1]) - inter)


def _random_boxes(rng, k, span=200.0):
    xy = rng.uniform(0, span, (k, 2))
    wh = rng.uniform(5, 60, (k, 2))
    return np.concatenate([xy, xy + wh], axis=1).astype(np.float32)


def test_iou_predicate_matches_fp64_away_from_threshold():
    rng = np.random.Generator(np.random.PCG64(404))
    a = _random_boxes(rng, 3000, 60)
    b = _random_boxes(rng, 3000, 60)
    got = post.iou_exceeds(a, b, 0.4)
    ref = np.array([_iou64(x.astype(float), y.astype(float)) for x, y in zip(a, b)])
    far = np.abs(ref - 0.4) > 1e-5
    assert far.sum() > 2900 and (ref > 0.4).sum() > 30
    np.testing.assert_array_equal(got[far], ref[far] > 0.4)
    # symmetric and identical boxes always exceed any thr < 1
    np.testing.assert_array_equal(post.iou_exceeds(b, a, 0.4), got)
    assert np.all(post.iou_exceeds(a, a, 0.999))


def check_greedy_nms_characterisation(boxes, margin, idx, thr, kept):
    """(i) kept is in (margin desc, idx asc) order; (ii) no two kept boxes overlap
    above thr; (iii) every suppressed box overlaps above thr with a kept box that
    precedes it.  These three properties determine greedy NMS uniquely."""
    order = list(post.sort_order(margin, idx))
    rank = {p: r for r, p in enumerate(order)}
    ranks = [rank[p] for p in kept]
    assert ranks == sorted(ranks)
    ks = set(int(p) for p in kept)
    for a in kept:
        for b in kept:
            if a != b:
                assert not post.iou_exceeds(boxes[a], boxes[b], thr)
    for p in order:
        if p in ks:
            continue
        assert any(rank[k] < rank[p] and post.iou_exceeds(boxes[k], boxes[p], thr) for k in kept)


@pytest.mark.parametrize("k,thr", [(0, 0.4), (1, 0.4), (60, 0.4), (300, 0.4), (200, 0.1), (200, 0.7)])
def test_nms_characterisation(k, thr):
    # a generator of its own (the session one's state depends on which tests ran
    # before on this worker), and an exact duplicate box (IoU 1): whatever the
    # draw, some box is suppressed at every threshold below 1
    rng = np.random.Generator(np.random.PCG64(7000 + 10 * k + int(round(100 * thr))))
    boxes = _random_boxes(rng, k)
    if k >= 2:
        boxes[k - 1] = boxes[0]
    margin = rng.normal(0, 2, k).astype(np.float32)
    margin[: k // 4] = margin[k // 2: k // 2 + k // 4]     # real ties, broken by idx
    idx = rng.permutation(10 * k + 1)[:k]
    kept = post.nms(boxes, margin, idx, thr)
    check_greedy_nms_characterisation(boxes, margin, idx, thr, list(kept))
    if k >= 60:
        assert 0 < len(kept) < k


def test_nms_special_cases(rng):
    boxes = _random_boxes(rng, 50)
    margin = rng.normal(0, 1, 50).astype(np.float32)
    idx = np.arange(50)
    assert len(post.nms(boxes, margin, idx, 1.0)) == 50           # IoU > 1 never holds
    same = np.repeat(boxes[:1], 7, axis=0)
    m = np.array([0.1, 0.5, 0.5, 0.2, 0.5, 0.0, 0.3], dtype=np.float32)
    kept = post.nms(same, m, np.array([9, 4, 2, 8, 3, 1, 7]), 0.4)
    assert list(kept) == [2]                                       # highest margin, lowest idx


def test_l2_normalize(rng):
    e = rng.standard_normal((20, 64)) * rng.uniform(1e-3, 1e3, (20, 1))
    u = post.l2_normalize(e)
    np.testing.assert_allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-12)
    cos = (u * e).sum(1) / np.linalg.norm(e, axis=1)
    np.testing.assert_allclose(cos, 1.0, atol=1e-12)
    assert np.all(post.l2_normalize(np.zeros((1, 8))) == 0.0)


def test_output_row_width_matches_paper():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["output_row"]
    dets = {"boxes": np.zeros((3, 4)), "score": np.zeros(3), "emb": np.zeros((3, g["embedding"])),
            "idx": np.arange(3)}
    rows = post.output_rows(dets)
    assert rows.shape == (3, g["total"]) == (3, g["box"] + g["objectness"] + g["class"] + g["embedding"])


def test_tiny_calibrated_candidate_count_and_pipeline():
    """beta_50 puts exactly 50 anchors over 0.5 on calibration frame 0 (FP64); the
    detections satisfy the NMS characterisation and have unit embeddings."""
    layers = model_weights(TINY, 50)
    out = net.forward(tiny_frame(TINY.seed, 0)[None], layers, TINY.blocks)
    d = post.detections(out, anchors_px(TINY), 0.5, 0.4)
    assert d["n_cand"] == 50
    c = post.decode_frame([x[0] for x in out["det"]], anchors_px(TINY), 0.5)
    pos = np.searchsorted(c["idx"], d["idx"])
    check_greedy_nms_characterisation(c["boxes"].astype(np.float32), c["margin"], c["idx"], 0.4, list(pos))
    np.testing.assert_allclose(np.linalg.norm(d["emb"], axis=1), 1.0, atol=1e-12)
    capped = post.detections(out, anchors_px(TINY), 0.5, 0.4, cap=10)
    assert capped["overflow"] and capped["n_cand"] == 50
    top = post.sort_order(c["margin"], c["idx"])[:10]
    assert set(capped["idx"]).issubset(set(c["idx"][top]))


def test_logit_offset_equals_shifted_foreground_logits(rng):
    """A per-frame offset d on c_fg is the same decode as c_fg + d written into
    the head outputs (the same FP32 add), and at threshold 0.5 it keeps exactly
    the anchors with c_fg - c_bg >= -d."""
    from oracle.post import decode_frame
    an = np.array([[[8.0, 24.0]] * 4, [[16.0, 48.0]] * 4, [[32.0, 96.0]] * 4], dtype=np.float32)
    det = [rng.normal(0, 2, (h, w, 24)).astype(np.float32) for h, w in ((6, 10), (3, 5), (2, 3))]
    d = np.float32(1.37)
    got = decode_frame(det, an, 0.5, logit_offset=float(d))
    shifted = [x.copy() for x in det]
    for x in shifted:
        x[..., 5::6] = x[..., 5::6] + d
    want = decode_frame(shifted, an, 0.5)
    np.testing.assert_array_equal(got["idx"], want["idx"])
    np.testing.assert_array_equal(got["margin"], want["margin"])
    n = sum(int(((x[..., 5::6] + d) - x[..., 4::6] >= 0).sum()) for x in det)
    assert len(got["idx"]) == n
    assert len(decode_frame(det, an, 0.5, logit_offset=-100.0)["idx"]) == 0
