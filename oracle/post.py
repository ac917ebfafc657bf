"""FP64 oracle of decode, threshold, sort, NMS and embedding normalisation.

Test infrastructure only.  Follows the post-processing list of Appendix A:
the model's per-detection row is 4 box values, an object confidence, a class
score and the embedding (item 1); detections whose score is below the
confidence threshold are discarded (item 2); the rest are sorted by score and
any detection whose IoU with a higher-scored kept detection is above the NMS
threshold is discarded (item 3).  Embeddings are compared by cosine distance
later (item 5), so they are L2-normalised here.

Readings where the paper is silent (anchor-relative decode "as in YOLOv3",
Sec. 3.1):

* per anchor a of a cell (i, j) at stride s, channels 6a + (dx, dy, dw, dh,
  c_bg, c_fg); score = 1 / (1 + exp(c_bg - c_fg)) (2-way softmax foreground);
  cx = (j + 1/2) s + dx aw, cy = (i + 1/2) s + dy ah,
  w = aw exp(min(dw, ln 64)), h = ah exp(min(dh, ln 64)); box not clipped.
* threshold: keep iff score >= thr, evaluated as the equivalent margin test
  (c_fg - c_bg) >= ln(thr / (1 - thr)) in the precision of the head outputs;
  at thr = 0.5 that is exactly c_fg >= c_bg.
* canonical index idx = base_s + A (i W_s + j) + a, scales ordered 8, 16, 32.
* sort by score descending, evaluated on the margin (a monotone function of
  the score that does not saturate), ties by idx ascending.
* NMS predicate: see ``iou_exceeds``.
* normalisation: e / max(||e||_2, 1e-12) of the emb map at the kept anchor's cell.
"""

import math

import numpy as np

CLIP = math.log(64.0)
NORM_EPS = 1e-12


def logit_threshold(thr, dtype=np.float64):
    """ln(thr / (1 - thr)), the margin equivalent of score >= thr."""
    thr = float(thr)
    if thr <= 0.0:
        return dtype(-np.inf)
    if thr >= 1.0:
        return dtype(np.inf)
    return dtype(math.log(thr / (1.0 - thr)))


def decode_frame(det_maps, anchors, thr, strides=(8, 16, 32), logit_offset=0.0):
    """Decode + threshold one frame.

    det_maps: list of [Hs, Ws, 6A] arrays (strides 8, 16, 32); anchors [3, A, 2] px.
    logit_offset: a per-frame confidence offset added to every foreground logit
    c_fg before the margin is formed (0: none).
    The margin test runs in the dtype of det_maps; box arithmetic in FP64.
    Returns dict of candidates in canonical-index order: idx (int64), margin
    (det dtype), score, boxes [K, 4] (x1, y1, x2, y2) FP64, and cell =
    (scale, i, j) per candidate.
    """
    dt = np.asarray(det_maps[0]).dtype.type
    lthr = logit_threshold(thr, dt)
    idx_l, mar_l, box_l, cell_l = [], [], [], []
    base = 0
    for si, (d, s) in enumerate(zip(det_maps, strides)):
        d = np.asarray(d)
        hs, ws, c = d.shape
        na = c // 6
        v = d.reshape(hs, ws, na, 6)
        cfg = v[..., 5] if logit_offset == 0.0 else v[..., 5] + dt(logit_offset)
        margin = cfg - v[..., 4]                          # in the head's precision
        keep = margin >= lthr
        ii, jj, aa = np.nonzero(keep)
        vv = v[ii, jj, aa].astype(np.float64)
        aw = anchors[si, aa, 0].astype(np.float64)
        ah = anchors[si, aa, 1].astype(np.float64)
        cx = (jj + 0.5) * s + vv[:, 0] * aw
        cy = (ii + 0.5) * s + vv[:, 1] * ah
        w = aw * np.exp(np.minimum(vv[:, 2], CLIP))
        h = ah * np.exp(np.minimum(vv[:, 3], CLIP))
        box_l.append(np.stack([cx - w / 2, cy - h / 2, cx + w / 2, cy + h / 2], axis=1))
        idx_l.append(base + na * (ii * ws + jj) + aa)
        mar_l.append(margin[ii, jj, aa])
        cell_l.append(np.stack([np.full_like(ii, si), ii, jj], axis=1))
        base += hs * ws * na
    idx = np.concatenate(idx_l).astype(np.int64)
    margin = np.concatenate(mar_l)
    order = np.argsort(idx, kind="stable")
    margin = margin[order]
    return {
        "idx": idx[order],
        "margin": margin,
        "score": 1.0 / (1.0 + np.exp(-margin.astype(np.float64))),
        "boxes": np.concatenate(box_l)[order].reshape(-1, 4),
        "cell": np.concatenate(cell_l)[order].reshape(-1, 3),
    }


def sort_order(margin, idx):
    """Permutation sorting by (margin descending, idx ascending)."""
    return np.lexsort((np.asarray(idx), -np.asarray(margin)))


def iou_exceeds(a, b, thr):
    """IoU(a, b) > thr, evaluated as inter > thr * uni in IEEE FP32.

    a: [4] or [K, 4] boxes (x1, y1, x2, y2), b likewise.  No +1 pixel
    convention.  Each operation is one correctly rounded FP32 op, in this order:
    iw = max(0, min(ax2, bx2) - max(ax1, bx1)); ih likewise; inter = iw * ih;
    area_a = (ax2 - ax1) * (ay2 - ay1); area_b likewise;
    uni = (area_a + area_b) - inter; result = inter > thr * uni.
    """
    f = np.float32
    a = np.asarray(a, dtype=f)
    b = np.asarray(b, dtype=f)
    t = f(thr)
    iw = np.maximum(f(0), np.minimum(a[..., 2], b[..., 2]) - np.maximum(a[..., 0], b[..., 0]))
    ih = np.maximum(f(0), np.minimum(a[..., 3], b[..., 3]) - np.maximum(a[..., 1], b[..., 1]))
    inter = iw * ih
    area_a = (a[..., 2] - a[..., 0]) * (a[..., 3] - a[..., 1])
    area_b = (b[..., 2] - b[..., 0]) * (b[..., 3] - b[..., 1])
    uni = (area_a + area_b) - inter
    return inter > t * uni


def nms(boxes, margin, idx, thr):
    """Greedy NMS (Appendix A, item 3).

    Sorts by (margin desc, idx asc); walks the list and keeps a box iff no
    already-kept box overlaps it with IoU > thr.  Returns positions (into the
    inputs) of the kept boxes, in keep order.
    """
    boxes = np.asarray(boxes, dtype=np.float32).reshape(-1, 4)
    order = sort_order(margin, idx)
    kept = []
    for p in order:
        if kept and np.any(iou_exceeds(boxes[kept], boxes[p], thr)):
            continue
        kept.append(int(p))
    return np.asarray(kept, dtype=np.int64)


def l2_normalize(e):
    """e / max(||e||_2, 1e-12), row-wise, FP64."""
    e = np.asarray(e, dtype=np.float64)
    n = np.sqrt((e * e).sum(axis=-1, keepdims=True))
    return e / np.maximum(n, NORM_EPS)


def detections(out, anchors, conf_thr=0.5, nms_thr=0.4, frame=0, cap=None, logit_offset=0.0):
    """Threshold -> sort -> NMS -> normalised embeddings for one frame.

    out: the forward's dict.  Returns dict with (in keep order) idx, margin,
    score, boxes (FP64), emb (FP64, unit rows), plus the pre-NMS candidate
    count 'n_cand' and 'overflow' when a candidate cap is given (the top ``cap``
    by (margin, idx) are kept).  ``logit_offset`` as in ``decode_frame``.
    """
    dets = [d[frame] for d in out["det"]]
    c = decode_frame(dets, anchors, conf_thr, logit_offset=logit_offset)
    n_cand = len(c["idx"])
    overflow = False
    if cap is not None and n_cand > cap:
        top = np.sort(sort_order(c["margin"], c["idx"])[:cap])
        c = {k: v[top] for k, v in c.items()}
        overflow = True
    keep = nms(c["boxes"], c["margin"], c["idx"], nms_thr)
    cells = c["cell"][keep]
    emb = np.stack([out["emb"][sc][frame][i, j] for sc, i, j in cells]) if len(keep) else \
        np.zeros((0, out["emb"][0].shape[-1]))
    return {
        "idx": c["idx"][keep], "margin": c["margin"][keep], "score": c["score"][keep],
        "boxes": c["boxes"][keep], "emb": l2_normalize(emb), "n_cand": n_cand,
        "overflow": overflow,
    }


def output_rows(dets):
    """The model-to-post row of Appendix A item 1: [x1, y1, x2, y2, score, class=0, emb...]."""
    n = len(dets["idx"])
    return np.concatenate([dets["boxes"], dets["score"][:, None], np.zeros((n, 1)), dets["emb"]], axis=1)
