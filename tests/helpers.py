"""Shared helpers of the tests (inputs, oracle runs, comparisons)."""

import functools

import numpy as np

from jde_inputs import TINY, FULL, model_weights, tiny_frame, scene_batch, anchors_px


def rel_err(got, ref):
    """Normwise max relative error max|g - r| / max|r| (per output tensor)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-30))


@functools.lru_cache(maxsize=None)
def weights(cfg_name, k):
    cfg = TINY if cfg_name == "tiny" else FULL
    return model_weights(cfg, k)


@functools.lru_cache(maxsize=None)
def frames(cfg_name, n, t0=0, h=None, w=None):
    cfg = TINY if cfg_name == "tiny" else FULL
    h = h or cfg.height
    w = w or cfg.width
    if cfg_name == "tiny":
        return np.stack([tiny_frame(cfg.seed, t0 + i, h, w) for i in range(n)])
    return scene_batch(cfg.seed, n, h, w, t0=t0)


@functools.lru_cache(maxsize=None)
def oracle_forward(cfg_name, k, n, t0=0, h=None, w=None):
    from oracle.network import forward
    cfg = TINY if cfg_name == "tiny" else FULL
    return forward(frames(cfg_name, n, t0, h, w), weights(cfg_name, k), cfg.blocks)


def head_views(heads, descs):
    """Per-frame [Hs, Ws, C] numpy views of packed GPU head outputs."""
    out = {"det": [], "emb": []}
    for key in ("det", "emb"):
        for s in range(3):
            flat = heads[key][s].cpu().numpy()
            st = 8 << s
            pix = [(h // st) * (w // st) for h, w in descs]
            c = flat.size // sum(pix)
            off = 0
            per = []
            for (h, w), p in zip(descs, pix):
                per.append(flat[off * c:(off + p) * c].reshape(h // st, w // st, c))
                off += p
            out[key].append(per)
    return out


def gpu_dets(d, f, cap):
    cnt = int(d["count"][f])
    sl = slice(f * cap, f * cap + cnt)
    return {k: d[k][sl].cpu().numpy() for k in ("boxes", "scores", "margins", "emb", "anchor_idx")} | {
        "n_cand": int(d["n_cand"][f]), "overflow": int(d["overflow"][f])}


def iou_matrix(a, b):
    a = np.asarray(a, np.float64)[:, None, :]
    b = np.asarray(b, np.float64)[None, :, :]
    iw = np.clip(np.minimum(a[..., 2], b[..., 2]) - np.maximum(a[..., 0], b[..., 0]), 0, None)
    ih = np.clip(np.minimum(a[..., 3], b[..., 3]) - np.maximum(a[..., 1], b[..., 1]), 0, None)
    inter = iw * ih
    ua = (a[..., 2] - a[..., 0]) * (a[..., 3] - a[..., 1]) + (b[..., 2] - b[..., 0]) * (b[..., 3] - b[..., 1]) - inter
    return inter / np.maximum(ua, 1e-30)


def match_fraction(gpu_boxes, ref_boxes, ref_order_scores, iou_min=0.9):
    """One-to-one greedy matching in reference-score order; fraction of reference
    detections matched by a GPU detection at IoU >= iou_min."""
    if len(ref_boxes) == 0:
        return 1.0, []
    if len(gpu_boxes) == 0:
        return 0.0, []
    m = iou_matrix(ref_boxes, gpu_boxes)
    used = set()
    pairs = []
    for r in np.argsort(-np.asarray(ref_order_scores), kind="stable"):
        cand = [(m[r, g], g) for g in range(m.shape[1]) if g not in used and m[r, g] >= iou_min]
        if cand:
            best = max(cand)[1]
            used.add(best)
            pairs.append((r, best))
    return len(pairs) / len(ref_boxes), pairs


def anchors(cfg_name):
    return anchors_px(TINY if cfg_name == "tiny" else FULL)


@functools.lru_cache(maxsize=None)
def oracle_forward_rounded(cfg_name, k, n, fmt):
    """Oracle forward of the network as stored in `fmt` ('bf16' or 'fp16'): conv
    weights rounded to the format (the stem stays FP32) and every stored
    activation rounded; arithmetic FP64."""
    from oracle.network import forward, round_bf16, round_fp16
    cfg = TINY if cfg_name == "tiny" else FULL
    rnd = round_bf16 if fmt == "bf16" else round_fp16
    layers = weights(cfg_name, k)
    layers = [layers[0]] + [(rnd(w), b) for w, b in layers[1:]]
    return forward(frames(cfg_name, n), layers, cfg.blocks, store=rnd)


def fp8_layer_set(cfg):
    """Convs that run in FP8: backbone 3x3 convs (after the stem) whose Cin % 128 == 0."""
    from jde_inputs import weight_specs
    n_backbone = 1 + 5 + 2 * sum(cfg.blocks)
    specs = weight_specs(cfg)
    return {i for i in range(1, n_backbone) if specs[i][2] == 3 and specs[i][3] % 128 == 0}


@functools.lru_cache(maxsize=None)
def oracle_forward_mx(cfg_name, k, n, fmt):
    """Oracle forward of the FP6 / FP4 network (a diagnostic: no test bound comes
    from it): as oracle_forward_fp8 with block scales, elements of ``fmt``."""
    from oracle.network import forward, round_bf16, quantize_blocks, quantize_per_channel_blocks
    cfg = TINY if cfg_name == "tiny" else FULL
    layers = weights(cfg_name, k)
    f8 = fp8_layer_set(cfg)
    lq = [layers[0]] + [(quantize_per_channel_blocks(w, fmt)[0] if i in f8 else round_bf16(w), b)
                        for i, (w, b) in enumerate(layers[1:], 1)]

    def quant(i, x):
        return quantize_blocks(x, fmt) if i in f8 else x

    return forward(frames(cfg_name, n), lq, cfg.blocks, store=round_bf16, in_hook=quant)


@functools.lru_cache(maxsize=None)
def oracle_forward_fp8(cfg_name, k, n, blocks=True):
    """Oracle forward of the FP8 network (a diagnostic: no test bound comes from it):
    BF16 storage and weights, and for each FP8 conv e4m3 weights with a per-channel
    scale and a power-of-two scale per 32-k block, and an e4m3 input with
    (blocks) a power-of-two scale per pixel and 32 channels or (not blocks) a
    static scale (max |x| of that input in the BF16 network on the same frames,
    / 448).  Returns (outputs, {conv index: static input scale})."""
    from oracle.network import (forward, round_bf16, round_fp8, quantize_fp8_blocks,
                                quantize_fp8_per_channel_blocks)
    cfg = TINY if cfg_name == "tiny" else FULL
    fr = frames(cfg_name, n)
    layers = weights(cfg_name, k)
    f8 = fp8_layer_set(cfg)
    lb = [layers[0]] + [(round_bf16(w), b) for w, b in layers[1:]]
    amax = {}

    def record(i, x):
        if i in f8:
            amax[i] = float(np.abs(x).max())
        return x

    forward(fr, lb, cfg.blocks, store=round_bf16, in_hook=record)
    scales = {i: (amax[i] / 448.0 if amax[i] > 0 else 1.0) for i in f8}
    lq = [(quantize_fp8_per_channel_blocks(layers[i][0])[0], b) if i in f8 else (w, b)
          for i, (w, b) in enumerate(lb)]

    def quant(i, x):
        if i not in f8:
            return x
        return quantize_fp8_blocks(x) if blocks else round_fp8(x / scales[i]) * scales[i]

    return forward(fr, lq, cfg.blocks, store=round_bf16, in_hook=quant), scales
