"""Python binding of libjde (argument marshalling only).

Every step of the hot path runs in the library's HIP kernels; torch tensors are
used only as device memory and the current HIP stream as the launch stream.
Function names follow the C ABI (include/jde.h).
"""

import ctypes

import numpy as np

from . import _lib
from ._lib import (JdeConfig, JdeFrameDesc, JdeHeadOut, JdeDets, check, load, load_host,  # noqa: F401
                   JDE_FP32, JDE_BF16, JDE_FP16, JDE_FP8, JDE_FP6, JDE_FP4)

PRECISIONS = {"fp32": JDE_FP32, "bf16": JDE_BF16, "fp16": JDE_FP16, "fp8": JDE_FP8, "fp6": JDE_FP6,
              "fp4": JDE_FP4}


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _descs(descs):
    arr = (JdeFrameDesc * len(descs))()
    for i, (h, w) in enumerate(descs):
        arr[i].h, arr[i].w = int(h), int(w)
    return arr


def jde_create(c0, blocks, emb_dim, anchors, precision="fp32", max_frames=1, max_h=608, max_w=1088,
               max_candidates=1024, max_pixels=0):
    """Create a context (host plan); returns an opaque handle (ctypes.c_void_p)."""
    lib = load()
    cfg = JdeConfig()
    cfg.base_ch = c0
    for i, b in enumerate(blocks):
        cfg.blocks[i] = b
    cfg.emb_dim = emb_dim
    cfg.num_anchors = 4
    an = np.asarray(anchors, dtype=np.float32).reshape(3, 4, 2)
    for s in range(3):
        for a in range(4):
            cfg.anchors[s][a][0] = float(an[s, a, 0])
            cfg.anchors[s][a][1] = float(an[s, a, 1])
    cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    cfg.max_frames = max_frames
    cfg.max_h = max_h
    cfg.max_w = max_w
    cfg.max_candidates = max_candidates
    cfg.max_pixels = int(max_pixels)
    h = ctypes.c_void_p()
    check(lib.jde_create(ctypes.byref(cfg), ctypes.byref(h)), "jde_create")
    return h


def jde_destroy(ctx):
    load().jde_destroy(ctx)


def jde_layer_info(ctx, i):
    co, k, ci, st = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(load().jde_layer_info(ctx, i, ctypes.byref(co), ctypes.byref(k), ctypes.byref(ci), ctypes.byref(st)),
          "jde_layer_info")
    return co.value, k.value, ci.value, st.value


def jde_cost_matrix(trk_emb, mean, cov, det_boxes, det_emb, gate=9.4877, cost=None, stream=None):
    """Device tensors in, [T, D] FP32 device cost out."""
    torch = _torch()
    T, E = trk_emb.shape
    D = det_boxes.shape[0]
    if cost is None:
        cost = torch.empty((T, D), dtype=torch.float32, device=trk_emb.device)
    check(load().jde_cost_matrix(_ptr(trk_emb), _ptr(mean), _ptr(cov), T, _ptr(det_boxes), _ptr(det_emb), D, E,
                                 float(gate), _ptr(cost), _stream(stream)), "jde_cost_matrix")
    return cost


def jde_ingest(src_u8, descs, out=None, stream=None):
    """8-bit RGB frames (device uint8 [n, H, W, 3]) -> packed NCHW FP32 model input
    at the sizes `descs` (letterbox + bilinear resize + /255)."""
    torch = _torch()
    n, H, W, C = src_u8.shape
    assert C == 3 and src_u8.dtype == torch.uint8 and src_u8.is_contiguous()
    total = sum(3 * h * w for h, w in descs)
    if out is None:
        out = torch.empty(total, dtype=torch.float32, device=src_u8.device)
    check(load().jde_ingest(_ptr(src_u8), int(n), int(H), int(W), _descs(descs), _ptr(out), _stream(stream)),
          "jde_ingest")
    return out


def jde_nms_noalloc(boxes, margins, idx, nms_iou=0.4, keep=None, nkeep=None, stream=None):
    """Greedy NMS of one candidate list on the library's static scratch (no
    workspace).  Device tensors in; keep positions [max(K, 1)] int32 and the
    kept count [1] int32 out (allocated here unless given)."""
    torch = _torch()
    K = int(boxes.shape[0])
    if keep is None:
        keep = torch.empty(max(K, 1), dtype=torch.int32, device=boxes.device)
    if nkeep is None:
        nkeep = torch.empty(1, dtype=torch.int32, device=boxes.device)
    check(load().jde_nms_noalloc(_ptr(boxes), _ptr(margins), _ptr(idx), K, float(nms_iou), _ptr(keep),
                                 _ptr(nkeep), _stream(stream)), "jde_nms_noalloc")
    return keep, nkeep


def jde_track_emb_update(pairs, det_emb, trk_emb, momentum=0.9, stream=None):
    P = pairs.shape[0]
    check(load().jde_track_emb_update(_ptr(pairs), P, _ptr(det_emb), det_emb.shape[0], _ptr(trk_emb),
                                      trk_emb.shape[0], trk_emb.shape[1], float(momentum), _stream(stream)),
          "jde_track_emb_update")
    return trk_emb


def _dets_of(dets, cap):
    """JdeDets struct of a dict of device tensors (missing entries -> NULL)."""
    ds = JdeDets()
    for k in ("boxes", "scores", "margins", "emb", "anchor_idx", "count", "n_cand", "overflow"):
        setattr(ds, k, dets[k].data_ptr() if k in dets else 0)
    ds.cap = int(cap)
    return ds


def _tb(track_begin):
    tb = np.ascontiguousarray(track_begin, dtype=np.int32)
    return tb, tb.ctypes.data_as(_lib.c_int_p)


def jde_cost_matrix_batch_fused(trk_emb, mean, cov, track_begin, dets, cap, motion_weight, gate=9.4877, cost=None,
                                stream=None):
    """Motion-fused batched cost [T, cap] (see jde_cost_matrix_batch_fused)."""
    torch = _torch()
    tb, tbp = _tb(track_begin)
    E = int(trk_emb.shape[1]) if trk_emb.dim() == 2 else int(dets["emb"].shape[-1])
    if cost is None:
        cost = torch.full((max(int(tb[-1]), 1), cap), float("nan"), dtype=torch.float32, device=dets["count"].device)
    ds = _dets_of(dets, cap)
    check(load().jde_cost_matrix_batch_fused(_ptr(trk_emb), _ptr(mean), _ptr(cov), tbp, ctypes.byref(ds),
                                             len(tb) - 1, E, float(gate), float(motion_weight), _ptr(cost),
                                             _stream(stream)), "jde_cost_matrix_batch_fused")
    return cost


def jde_iou_cost_batch(mean, track_begin, dets, cap, cost=None, stream=None):
    """Box-overlap cost [T, cap] = 1 - IoU(track box from its state, detection box)."""
    torch = _torch()
    tb, tbp = _tb(track_begin)
    if cost is None:
        cost = torch.full((max(int(tb[-1]), 1), cap), float("nan"), dtype=torch.float32, device=dets["count"].device)
    ds = _dets_of(dets, cap)
    check(load().jde_iou_cost_batch(_ptr(mean), tbp, ctypes.byref(ds), len(tb) - 1, _ptr(cost), _stream(stream)),
          "jde_iou_cost_batch")
    return cost


def jde_kf_predict_dev(mean, cov, stream=None):
    """Device Kalman predict in place: mean [T, 8], cov [T, 8, 8] FP64 device tensors."""
    T = int(mean.shape[0])
    check(load().jde_kf_predict_dev(T, _ptr(mean), _ptr(cov), _stream(stream)), "jde_kf_predict_dev")
    return mean, cov


def jde_kf_update_dev(track_begin, det_of_track, dets, cap, mean, cov, status=None, stream=None):
    """Device Kalman update of each track with its assigned detection box (batched layout)."""
    tb, tbp = _tb(track_begin)
    ds = _dets_of(dets, cap)
    check(load().jde_kf_update_dev(tbp, len(tb) - 1, _ptr(det_of_track), ctypes.byref(ds), _ptr(mean), _ptr(cov),
                                   _ptr(status), _stream(stream)), "jde_kf_update_dev")
    return mean, cov


def jde_assign_dev(cost, track_begin, dets, cap, max_cost, out=None, stream=None):
    """Device min-cost assignment of every frame of a batched cost [T, cap];
    returns dict of device tensors det_of_track [T], track_of_det [n*cap], kept [n],
    total [n] (FP64), status [n]."""
    torch = _torch()
    tb, tbp = _tb(track_begin)
    n = len(tb) - 1
    dev = dets["count"].device
    if out is None:
        out = {"det_of_track": torch.empty(max(int(tb[-1]), 1), dtype=torch.int32, device=dev),
               "track_of_det": torch.empty(max(n * cap, 1), dtype=torch.int32, device=dev),
               "kept": torch.empty(max(n, 1), dtype=torch.int32, device=dev),
               "total": torch.empty(max(n, 1), dtype=torch.float64, device=dev),
               "status": torch.empty(max(n, 1), dtype=torch.int32, device=dev)}
    ds = _dets_of(dets, cap)
    check(load().jde_assign_dev(_ptr(cost), tbp, n, ctypes.byref(ds), float(max_cost), _ptr(out["det_of_track"]),
                                _ptr(out["track_of_det"]), _ptr(out["kept"]), _ptr(out["total"]), _ptr(out["status"]),
                                _stream(stream)), "jde_assign_dev")
    return out


def jde_kf_initiate(z):
    mean = np.zeros(8)
    cov = np.zeros(64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    load_host().jde_kf_initiate(z.ctypes.data_as(_lib.c_double_p), mean.ctypes.data_as(_lib.c_double_p),
                           cov.ctypes.data_as(_lib.c_double_p))
    return mean, cov.reshape(8, 8)


def jde_kf_initiate_n(zs):
    """zs [n, 4] -> (mean [n, 8], cov [n, 8, 8])."""
    z = np.ascontiguousarray(zs, dtype=np.float64).reshape(-1, 4)
    n = z.shape[0]
    mean = np.zeros((n, 8))
    cov = np.zeros((n, 8, 8))
    load_host().jde_kf_initiate_n(n, z.ctypes.data_as(_lib.c_double_p), mean.ctypes.data_as(_lib.c_double_p),
                             cov.ctypes.data_as(_lib.c_double_p))
    return mean, cov


def jde_kf_predict(mean, cov):
    """In place on contiguous FP64 arrays [T, 8], [T, 8, 8]."""
    assert mean.dtype == np.float64 and cov.dtype == np.float64 and mean.flags.c_contiguous and cov.flags.c_contiguous
    load_host().jde_kf_predict(mean.shape[0], mean.ctypes.data_as(_lib.c_double_p), cov.ctypes.data_as(_lib.c_double_p))
    return mean, cov


def jde_kf_update(mean, cov, z):
    mean = np.ascontiguousarray(mean, dtype=np.float64).copy()
    cov = np.ascontiguousarray(cov, dtype=np.float64).copy()
    z = np.ascontiguousarray(z, dtype=np.float64)
    check(load_host().jde_kf_update(mean.ctypes.data_as(_lib.c_double_p), cov.ctypes.data_as(_lib.c_double_p),
                               z.ctypes.data_as(_lib.c_double_p)), "jde_kf_update")
    return mean, cov


def jde_kf_update_n(track_idx, det_idx, mean, cov, z):
    """Batched update in place: mean [T, 8] / cov [T, 8, 8] (contiguous FP64) rows
    track_idx[i] take z[det_idx[i]] (z [D, 4])."""
    assert mean.dtype == np.float64 and cov.dtype == np.float64 and mean.flags.c_contiguous and cov.flags.c_contiguous
    ti = np.ascontiguousarray(track_idx, dtype=np.int32)
    di = np.ascontiguousarray(det_idx, dtype=np.int32)
    z = np.ascontiguousarray(z, dtype=np.float64)
    assert ti.shape == di.shape and ti.ndim == 1
    if len(ti):
        assert 0 <= ti.min() and ti.max() < mean.shape[0] and 0 <= di.min() and di.max() < z.shape[0]
    check(load_host().jde_kf_update_n(len(ti), ti.ctypes.data_as(_lib.c_int_p), di.ctypes.data_as(_lib.c_int_p),
                                 mean.ctypes.data_as(_lib.c_double_p), cov.ctypes.data_as(_lib.c_double_p),
                                 z.ctypes.data_as(_lib.c_double_p)), "jde_kf_update_n")
    return mean, cov


def jde_box_to_z(boxes):
    """Host boxes [n, 4] (x1, y1, x2, y2) -> Kalman measurements [n, 4] FP64 (cx, cy, w/h, h)."""
    b = np.ascontiguousarray(boxes, dtype=np.float32).reshape(-1, 4)
    z = np.zeros((b.shape[0], 4))
    load_host().jde_box_to_z(b.shape[0], b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                             z.ctypes.data_as(_lib.c_double_p))
    return z


def jde_fp8_encode(x):
    """Host OCP e4m3 encoding (RNE, saturating) of a float array -> uint8 codes."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.zeros(x.shape, dtype=np.uint8)
    load_host().jde_fp8_encode(x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), x.size)
    return out


def jde_mx_encode(fmt, x):
    """Host FP6 E2M3 (fmt 'fp6') / FP4 E2M1 (fmt 'fp4') encoding (RNE, saturating)
    of a float array -> one code per uint8."""
    f = {"fp6": 2, "fp4": 4}[fmt]
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.zeros(x.shape, dtype=np.uint8)
    load_host().jde_mx_encode(f, x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), x.size)
    return out


def jde_assign(cost, max_cost):
    """Host cost [T, D] -> (pairs [P, 2] (t, d) sorted by t, total)."""
    c = np.ascontiguousarray(cost, dtype=np.float32)
    T, D = c.shape
    dot = np.full(max(T, 1), -1, dtype=np.int32)
    tod = np.full(max(D, 1), -1, dtype=np.int32)
    tot = ctypes.c_double()
    k = load_host().jde_assign(c.ctypes.data_as(_lib.c_float_p), T, D, float(max_cost),
                          dot.ctypes.data_as(_lib.c_int_p), tod.ctypes.data_as(_lib.c_int_p), ctypes.byref(tot))
    if k < 0:
        check(k, "jde_assign")
    t = np.nonzero(dot[:T] >= 0)[0]
    pairs = np.stack([t, dot[t].astype(np.int64)], axis=1) if T else np.zeros((0, 2), dtype=np.int64)
    return pairs, tot.value


class JDE:
    """A context plus the device buffers it needs (weights, workspace).

    `layers` for load_weights is the blob-order list of (w [Cout,k,k,Cin], b [Cout]) FP32 arrays.
    """

    def __init__(self, c0, blocks, emb_dim, anchors, precision="fp32", max_frames=1, max_h=608, max_w=1088,
                 max_candidates=1024, device="cuda", max_pixels=0):
        torch = _torch()
        self.lib = load()
        self.ctx = jde_create(c0, blocks, emb_dim, anchors, precision, max_frames, max_h, max_w, max_candidates,
                              max_pixels)
        self.E = emb_dim
        self.cap = max_candidates
        self.max_frames, self.max_h, self.max_w = max_frames, max_h, max_w
        self.device = torch.device(device)
        self.weights = torch.empty(self.lib.jde_weights_bytes(self.ctx), dtype=torch.uint8, device=self.device)
        self.ws = torch.empty(self.lib.jde_workspace_bytes(self.ctx), dtype=torch.uint8, device=self.device)

    def __del__(self):
        try:
            if getattr(self, "ctx", None) is not None:
                self.lib.jde_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def num_layers(self):
        return self.lib.jde_num_layers(self.ctx)

    def layer_shapes(self):
        return [jde_layer_info(self.ctx, i) for i in range(self.num_layers())]

    def load_weights(self, layers, stream=None):
        blob = np.concatenate([np.concatenate([np.asarray(w, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                               for w, b in layers])
        blob = np.ascontiguousarray(blob, dtype=np.float32)
        check(self.lib.jde_load_weights(self.ctx, blob.ctypes.data_as(_lib.c_float_p), blob.size,
                                        _ptr(self.weights), self.weights.numel(), _stream(stream)),
              "jde_load_weights")

    def head_buffers(self, descs, emb=True):
        """Head output buffers; emb=False leaves the dense embedding maps out (sparse emb head)."""
        torch = _torch()
        d = _descs(descs)
        det = (ctypes.c_size_t * 3)()
        embn = (ctypes.c_size_t * 3)()
        check(self.lib.jde_head_sizes(self.ctx, d, len(descs), det, embn), "jde_head_sizes")
        return {"det": [torch.empty(det[s], dtype=torch.float32, device=self.device) for s in range(3)],
                "emb": [torch.empty(embn[s], dtype=torch.float32, device=self.device) if emb else None
                        for s in range(3)]}

    def _head_struct(self, heads):
        h = JdeHeadOut()
        for s in range(3):
            h.det[s] = heads["det"][s].data_ptr()
            h.emb[s] = heads["emb"][s].data_ptr() if heads["emb"][s] is not None else 0
        return h

    def sparse_emb(self, on=True):
        """Deferred sparse embedding head (jde_sparse_emb)."""
        check(self.lib.jde_sparse_emb(self.ctx, int(on)), "jde_sparse_emb")

    def forward(self, frames, descs=None, heads=None, stream=None):
        """frames: contiguous FP32 device tensor, [n, 3, H, W] or packed 1-D with `descs`."""
        if descs is None:
            n, _, H, W = frames.shape
            descs = [(H, W)] * n
        if heads is None:
            heads = self.head_buffers(descs)
        hs = self._head_struct(heads)
        check(self.lib.jde_forward(self.ctx, _ptr(frames), _descs(descs), len(descs), _ptr(self.ws),
                                   self.ws.numel(), ctypes.byref(hs), _stream(stream)), "jde_forward")
        return heads

    def dets_buffers(self, n):
        torch = _torch()
        f32 = dict(dtype=torch.float32, device=self.device)
        i32 = dict(dtype=torch.int32, device=self.device)
        return {"boxes": torch.empty((n * self.cap, 4), **f32), "scores": torch.empty(n * self.cap, **f32),
                "margins": torch.empty(n * self.cap, **f32), "emb": torch.empty((n * self.cap, self.E), **f32),
                "anchor_idx": torch.empty(n * self.cap, **i32), "count": torch.empty(n, **i32),
                "n_cand": torch.empty(n, **i32), "overflow": torch.empty(n, **i32)}

    def _dets_struct(self, dets):
        ds = JdeDets()
        for k in ("boxes", "scores", "margins", "emb", "anchor_idx", "count", "n_cand", "overflow"):
            setattr(ds, k, dets[k].data_ptr())
        ds.cap = self.cap
        return ds

    def decode(self, heads, descs, conf_thr=0.5, nms_iou=0.4, dets=None, stream=None, logit_offset=None):
        """logit_offset: device FP32 [n] added to every c_fg of frame f, or None."""
        if dets is None:
            dets = self.dets_buffers(len(descs))
        if logit_offset is not None:
            assert logit_offset.dtype == _torch().float32 and logit_offset.numel() >= len(descs)
        ds = self._dets_struct(dets)
        hs = self._head_struct(heads)
        check(self.lib.jde_decode(self.ctx, ctypes.byref(hs), _descs(descs), len(descs), float(conf_thr),
                                  float(nms_iou), _ptr(logit_offset), _ptr(self.ws), self.ws.numel(),
                                  ctypes.byref(ds), _stream(stream)), "jde_decode")
        return dets

    def frame_bytes(self, h, w):
        """Device bytes one h x w frame occupies while in flight (jde_frame_bytes)."""
        return int(self.lib.jde_frame_bytes(self.ctx, int(h), int(w)))

    def admit(self, descs, in_flight_bytes, budget_bytes):
        """Number of leading frames of `descs` the device-memory budget admits (0 when
        the budget refuses the first one: JDE_EBUDGET)."""
        n = ctypes.c_int(0)
        st = self.lib.jde_admit(self.ctx, _descs(descs), len(descs), int(in_flight_bytes), int(budget_bytes),
                                ctypes.byref(n))
        if st == _lib.JDE_EBUDGET:
            return 0
        check(st, "jde_admit")
        return n.value

    def nms(self, boxes, margins, idx, nms_iou=0.4, stream=None):
        torch = _torch()
        K = int(boxes.shape[0])
        keep = torch.empty(max(K, 1), dtype=torch.int32, device=self.device)
        nkeep = torch.empty(1, dtype=torch.int32, device=self.device)
        check(self.lib.jde_nms(self.ctx, _ptr(boxes), _ptr(margins), _ptr(idx), K, float(nms_iou), _ptr(self.ws),
                               self.ws.numel(), _ptr(keep), _ptr(nkeep), _stream(stream)), "jde_nms")
        return keep, nkeep

    def cost_dets(self, trk_emb, mean, cov, dets, frame, gate=9.4877, cost=None, stream=None):
        """Cost of tracks against frame `frame` of a decode result; [T, cap] FP32 (columns
        >= count[frame] untouched)."""
        torch = _torch()
        T = int(trk_emb.shape[0])
        if cost is None:
            cost = torch.empty((T, self.cap), dtype=torch.float32, device=self.device)
        ds = self._dets_struct(dets)
        check(self.lib.jde_cost_matrix_dets(_ptr(trk_emb), _ptr(mean), _ptr(cov), T, ctypes.byref(ds), int(frame),
                                            self.E, float(gate), _ptr(cost), _stream(stream)),
              "jde_cost_matrix_dets")
        return cost

    def cost_batch(self, trk_emb, mean, cov, track_begin, dets, gate=9.4877, cost=None, stream=None):
        """Cost of every frame of a decode result against its own track range
        [track_begin[f], track_begin[f+1]); [track_begin[-1], cap] FP32."""
        torch = _torch()
        tb = np.ascontiguousarray(track_begin, dtype=np.int32)
        n = tb.size - 1
        if cost is None:
            cost = torch.empty((int(tb[-1]), self.cap), dtype=torch.float32, device=self.device)
        ds = self._dets_struct(dets)
        check(self.lib.jde_cost_matrix_batch(_ptr(trk_emb), _ptr(mean), _ptr(cov), tb.ctypes.data_as(_lib.c_int_p),
                                             ctypes.byref(ds), n, self.E, float(gate), _ptr(cost), _stream(stream)),
              "jde_cost_matrix_batch")
        return cost

    def autotune(self, frames, descs=None, heads=None, reps=3, stream=None):
        """Pick each convolution's tile by timing on this batch; returns the choices."""
        if descs is None:
            n, _, H, W = frames.shape
            descs = [(H, W)] * n
        if heads is None:
            heads = self.head_buffers(descs)
        hs = self._head_struct(heads)
        check(self.lib.jde_autotune(self.ctx, _ptr(frames), _descs(descs), len(descs), _ptr(self.ws),
                                    self.ws.numel(), ctypes.byref(hs), int(reps), _stream(stream)), "jde_autotune")
        return self.tiles()

    def _n_ops(self):
        n = ctypes.c_int()
        check(self.lib.jde_profile_collect(self.ctx, 0, None, None, None, ctypes.byref(n), None),
              "jde_profile_collect")
        return n.value

    def tiles(self):
        t = np.zeros(self._n_ops(), dtype=np.int32)
        check(self.lib.jde_tiles(self.ctx, t.ctypes.data_as(_lib.c_int_p), t.size, 0), "jde_tiles")
        return t

    def set_tiles(self, tiles):
        t = np.ascontiguousarray(tiles, dtype=np.int32)
        check(self.lib.jde_tiles(self.ctx, t.ctypes.data_as(_lib.c_int_p), t.size, 1), "jde_tiles")

    def graph_capture(self, frames, descs, heads, dets, conf_thr=0.5, nms_iou=0.4, tracks=None, cost=None,
                      stream=None, logit_offset=None):
        """Capture forward + decode (+ batched cost when tracks = (trk_emb, mean, cov, track_begin))
        on `stream` (a torch.cuda.Stream, not the default stream); returns a Graph."""
        hs = self._head_struct(heads)
        ds = self._dets_struct(dets)
        tb = None
        fe = mean = cov = None
        if tracks is not None:
            fe, mean, cov, track_begin = tracks
            tb = np.ascontiguousarray(track_begin, dtype=np.int32)
        g = ctypes.c_void_p()
        check(self.lib.jde_graph_capture(self.ctx, _ptr(frames), _descs(descs), len(descs), _ptr(self.ws),
                                         self.ws.numel(), ctypes.byref(hs), float(conf_thr), float(nms_iou),
                                         _ptr(logit_offset), ctypes.byref(ds), _ptr(fe), _ptr(mean), _ptr(cov),
                                         None if tb is None else tb.ctypes.data_as(_lib.c_int_p), _ptr(cost),
                                         _stream(stream), ctypes.byref(g)), "jde_graph_capture")
        return Graph(self.lib, g, (frames, heads, dets, tracks, cost, tb, logit_offset))

    def graph_capture_any(self, frames, heads, dets, conf_thr=0.5, nms_iou=0.4, stream=None, logit_offset=None):
        """One graph of forward + decode for any batch within the capacity
        (jde_graph_capture_any); replay with Graph.launch_batch(descs)."""
        hs = self._head_struct(heads)
        ds = self._dets_struct(dets)
        g = ctypes.c_void_p()
        check(self.lib.jde_graph_capture_any(self.ctx, _ptr(frames), _ptr(self.ws), self.ws.numel(),
                                             ctypes.byref(hs), float(conf_thr), float(nms_iou), _ptr(logit_offset),
                                             ctypes.byref(ds), _stream(stream), ctypes.byref(g)),
              "jde_graph_capture_any")
        return Graph(self.lib, g, (frames, heads, dets, logit_offset, self.ws))

    def capacity_descs(self):
        """The largest batch of the context as frame sizes (for sizing buffers)."""
        return [(self.max_h, self.max_w)] * self.max_frames

    def fp8_block_scales(self, on=True):
        """FP8 contexts: per-pixel, per-32-channel E8M0 activation scales (on, the
        default) or static per-tensor scales from ``calibrate`` (off)."""
        check(self.lib.jde_fp8_block_scales(self.ctx, int(bool(on))), "jde_fp8_block_scales")

    def calibrate(self, frames, descs=None, heads=None, stream=None):
        """FP8 contexts: set the static per-tensor activation scales (used with block
        scales off) from one BF16 forward of this batch."""
        if descs is None:
            n, _, H, W = frames.shape
            descs = [(H, W)] * n
        if heads is None:
            heads = self.head_buffers(descs)
        hs = self._head_struct(heads)
        check(self.lib.jde_calibrate(self.ctx, _ptr(frames), _descs(descs), len(descs), _ptr(self.ws),
                                     self.ws.numel(), ctypes.byref(hs), _stream(stream)), "jde_calibrate")
        return self.fp8_scales()

    def fp8_scales(self):
        out = np.zeros(self._n_ops(), dtype=np.float32)
        check(self.lib.jde_fp8_scales(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), out.size),
              "jde_fp8_scales")
        return out

    def fuse_stem(self, on=True):
        """Run the stem and the first downsample conv as one launch (16-bit only)."""
        check(self.lib.jde_fuse_stem(self.ctx, 1 if on else 0), "jde_fuse_stem")

    def fuse_blocks(self, on=True):
        """Run each 64- and 128-channel residual block as one launch (16-bit only)."""
        check(self.lib.jde_fuse_blocks(self.ctx, 1 if on else 0), "jde_fuse_blocks")

    def fold_det(self, on=True):
        """Run each head's det 1x1 in its det 3x3's epilogue (16-bit only)."""
        check(self.lib.jde_fold_det(self.ctx, 1 if on else 0), "jde_fold_det")

    def window_down(self, on=True):
        """Run the 3x3 stride-2 downsample convs with Cin 64 from an LDS window (16-bit only)."""
        check(self.lib.jde_window_down(self.ctx, 1 if on else 0), "jde_window_down")

    def window_convs(self, on=True):
        """Run qualifying 3x3 stride-1 convs from an LDS window (16-bit only)."""
        check(self.lib.jde_window_convs(self.ctx, 1 if on else 0), "jde_window_convs")

    def profile_begin(self, on=True):
        check(self.lib.jde_profile_begin(self.ctx, 1 if on else 0), "jde_profile_begin")

    def profile_collect(self):
        """(op_ms summed over profiled forwards, op_flop per launch, op_kind, n_forwards)."""
        n = self.num_layers() + 8
        ms = np.zeros(n)
        fl = np.zeros(n)
        kind = np.zeros(n, dtype=np.int32)
        nops = ctypes.c_int()
        nfwd = ctypes.c_int()
        check(self.lib.jde_profile_collect(self.ctx, n, ms.ctypes.data_as(_lib.c_double_p),
                                           fl.ctypes.data_as(_lib.c_double_p), kind.ctypes.data_as(_lib.c_int_p),
                                           ctypes.byref(nops), ctypes.byref(nfwd)), "jde_profile_collect")
        k = nops.value
        return ms[:k], fl[:k], kind[:k], nfwd.value


class Graph:
    """A captured step; keeps the captured buffers alive."""

    def __init__(self, lib, handle, keep):
        self.lib = lib
        self.h = handle
        self._keep = keep

    def launch_batch(self, descs, stream=None):
        """Replays a graph of graph_capture_any for the batch `descs` (frame sizes)."""
        check(self.lib.jde_graph_launch_batch(self.h, _descs(descs), len(descs), _stream(stream)),
              "jde_graph_launch_batch")

    def launch(self, stream=None):
        check(self.lib.jde_graph_launch(self.h, _stream(stream)), "jde_graph_launch")

    def __del__(self):
        try:
            if self.h:
                self.lib.jde_graph_destroy(self.h)
                self.h = None
        except Exception:
            pass
