"""Serving loop: concurrent video streams through the JDE hot path.

The paper's updated pipeline (Sec. 4.4) runs model prediction on batches of
frames while a separate post-processing worker consumes the model's outputs
and does the association (Appendix A items 4-9), so the forward never waits for
post-processing (Sec. 4.3).  This module is that pipeline for one GPU:

* frames of several streams arrive in real time (each stream at its own frame
  rate and resolution); they wait in arrival order;
* continuous batching: whenever a batch slot is free, every waiting frame that
  fits is admitted -- at most `max_batch` frames, and only while the frames in
  flight stay within the device-memory budget (the library's jde_admit, which
  charges each frame its pixels, head outputs, detection rows and workspace
  share); frames of different resolutions share one ragged batch;
* each stream has its own density of objects; its frames carry a confidence
  offset (the library's per-frame logit offset) that sets its candidates per
  frame;
* each slot owns a library context (workspace, head and detection buffers), a
  HIP stream and one captured graph of forward + decode that serves any ragged
  batch of the slot (replayed with the batch's frame table); its work overlaps
  the other slot's;
* a post-processing thread takes finished batches in order and, per frame in
  stream order, runs the association (Appendix A items 4-9).  With
  device_assoc (the default) every track's Kalman state and embedding live in
  device pools: Kalman predict, the gated cost matrix, the assignment and the
  Kalman update run on the GPU (the library's FP64 kernels, bit-identical to
  its host calls), and the host only reads back each track's matched
  detection for the track lifecycle (ids, lost counts, new tracks).  Without
  it the Kalman filter and the assignment run on the host in FP64 and only the
  cost matrix and the embeddings are on the device;
* latency of a frame = its arrival time -> its tracks updated.

Everything on the device runs in the library's kernels; this module only
schedules and marshals.
"""

import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from ._lib import JdeError
from .jde import (JDE, jde_kf_initiate_n, jde_kf_predict, jde_kf_update_n, jde_assign,
                  jde_track_emb_update, jde_box_to_z, jde_kf_predict_dev, jde_kf_update_dev, jde_assign_dev)

CHI2_GATE = 9.4877


@dataclass
class StreamSpec:
    sid: int
    height: int
    width: int
    fps: float
    phase: float                 # seconds after start of frame 0
    frames: np.ndarray           # [F, 3, H, W] FP32 host frames, played forward then backward
    logit_offset: float = 0.0    # added to every c_fg of the stream's frames (its density)
    n_obj: int = 0               # objects in the stream's scene

    def frame_index(self, t):
        """Frame t of the stream: the F rendered frames played 0..F-1, F-2..1, 0.. so
        that objects keep moving continuously (they reverse at the ends)."""
        F = len(self.frames)
        if F <= 1:
            return 0
        k = t % (2 * F - 2)
        return k if k < F else 2 * F - 2 - k


@dataclass
class StreamState:
    """Tracks of one stream as arrays (row k = one track): host FP64 Kalman state,
    ids, frames lost, and the track's row in the device embedding pool."""
    spec: StreamSpec
    pinned: list = field(default_factory=list)     # the stream's frames in pinned host memory
    mean: np.ndarray = None                        # [T, 8]
    cov: np.ndarray = None                         # [T, 8, 8]
    ids: np.ndarray = None                         # [T] int64
    lost: np.ndarray = None                        # [T] int64
    rows: np.ndarray = None                        # [T] int64 rows of the pool
    free_rows: list = field(default_factory=list)  # free rows of this stream's range of the pool
    next_id: int = 1

    def __post_init__(self):
        self.mean = np.zeros((0, 8))
        self.cov = np.zeros((0, 8, 8))
        self.ids = np.zeros(0, dtype=np.int64)
        self.lost = np.zeros(0, dtype=np.int64)
        self.rows = np.zeros(0, dtype=np.int64)


@dataclass
class FrameJob:
    sid: int
    t: int                       # frame index within its stream
    arrival: float
    admitted: float = 0.0


class Server:
    def __init__(self, cfg, anchors, layers, streams, precision="bf16", max_batch=16, hbm_budget=None,
                 max_tracks=512, max_cost=0.7, max_lost=30, conf_thr=0.5, nms_iou=0.4, cap=512, tiles=None,
                 device="cuda", device_assoc=True, sparse_emb=True, use_graph=True):
        import torch
        self.torch = torch
        self.device_assoc = device_assoc
        self.streams = {s.sid: StreamState(s) for s in streams}
        self.max_batch = max_batch
        self.max_cost, self.max_lost = max_cost, max_lost
        self.conf_thr, self.nms_iou = conf_thr, nms_iou
        self.E = cfg.emb_dim
        max_h = max(s.height for s in streams)
        max_w = max(s.width for s in streams)
        self.slots = []
        for _ in range(2):
            m = JDE(cfg.c0, cfg.blocks, cfg.emb_dim, anchors, precision, max_batch, max_h, max_w, cap, device)
            m.load_weights(layers)
            m.sparse_emb(sparse_emb)
            if tiles is not None:
                m.set_tiles(tiles)
            self.slots.append({"m": m, "stream": torch.cuda.Stream(), "busy": False})
        # Admission by device-memory budget: each frame in flight is charged what the
        # library says it occupies (pixels, heads, detection rows, workspace share).
        # The default budget is what the two slots can hold at once.
        m0 = self.slots[0]["m"]
        self.hbm_budget = int(hbm_budget) if hbm_budget is not None else 2 * max_batch * m0.frame_bytes(max_h, max_w)
        self.in_flight_bytes = 0
        self.budget_stalls = 0           # free slot and waiting frames, but the budget admitted none
        self.budget_cut = 0              # batches the budget cut below what was waiting (and max_batch)
        self.post_stream = torch.cuda.Stream()
        # Device-resident track embeddings of every stream in one pool: stream k owns
        # rows [k * max_tracks, (k + 1) * max_tracks).
        self.pool = torch.zeros((len(self.streams) * max_tracks, self.E), dtype=torch.float32, device=device)
        # ... and, with device_assoc, their Kalman states (FP64), same rows
        if device_assoc:
            self.kmean = torch.zeros((len(self.streams) * max_tracks, 8), dtype=torch.float64, device=device)
            self.kcov = torch.zeros((len(self.streams) * max_tracks, 8, 8), dtype=torch.float64, device=device)
        for k, st in enumerate(self.streams.values()):
            st.free_rows = list(range(k * max_tracks, (k + 1) * max_tracks))[::-1]
        # Frames arrive in pinned host memory (where a capture process would write
        # them); each admitted frame is one async H2D copy into its slot's buffer.
        for st in self.streams.values():
            st.pinned = [torch.from_numpy(np.ascontiguousarray(f).ravel()).pin_memory() for f in st.spec.frames]
        self.max_pix = max_batch * max_h * max_w * 3
        self.t_launch = 0.0
        self.t_post = 0.0
        self.t_parts = {"predict": 0.0, "cost": 0.0, "host_assoc": 0.0, "assign_update": 0.0,
                        "assign_update_cpu": 0.0, "lifecycle": 0.0, "update_sync": 0.0, "tracks": 0,
                        "frames": 0}
        for sl in self.slots:
            sl["dev"] = torch.empty(self.max_pix, dtype=torch.float32, device=device)
            # per-frame confidence offsets: written on the host, copied with the frames (the
            # slot's previous copy has completed before the slot is free again)
            sl["off_host"] = torch.zeros(max_batch, dtype=torch.float32).pin_memory()
            sl["off"] = torch.zeros(max_batch, dtype=torch.float32, device=device)
            # outputs sized for a full batch of the largest frames; smaller batches use a prefix
            sl["heads"] = sl["m"].head_buffers([(max_h, max_w)] * max_batch, emb=not sparse_emb)
            sl["dets"] = sl["m"].dets_buffers(max_batch)
            # one graph of forward + decode for any ragged batch of the slot (BF16 / FP16 contexts
            # with the fused stem; others launch eagerly)
            sl["graph"] = None
            if use_graph:
                try:
                    sl["graph"] = sl["m"].graph_capture_any(sl["dev"], sl["heads"], sl["dets"], conf_thr, nms_iou,
                                                            stream=sl["stream"], logit_offset=sl["off"])
                except JdeError:
                    sl["graph"] = None
        torch.cuda.synchronize()
        self.lock = threading.Lock()
        self.results = []            # per frame: dict(sid, t, boxes, ids, latency)
        self.cand = {sid: [] for sid in self.streams}   # candidates per frame, per stream

    def calibrate_density(self, iters=28):
        """Sets each stream's confidence offset so that its first frame gives as many
        candidates (anchors over the threshold, before NMS) as the stream has
        objects: the library decodes the frame at trial offsets, and a bisection on
        its candidate count finds the offsets o_K and o_K+1 at which the count first
        reaches K and K + 1; the stream gets their midpoint (the threshold then sits
        mid-gap between the K-th and (K+1)-th margin)."""
        torch = self.torch
        m = self.slots[0]["m"]
        heads, dets = self.slots[0]["heads"], self.slots[0]["dets"]
        off = self.slots[0]["off"][:1]

        def count(o, desc):
            off.fill_(o)
            m.decode(heads, [desc], self.conf_thr, self.nms_iou, dets=dets, logit_offset=off)
            return int(dets["n_cand"][0].item())

        def first_reaching(k, desc, lo=-40.0, hi=40.0):
            for _ in range(iters):
                mid = 0.5 * (lo + hi)
                if count(mid, desc) >= k:
                    hi = mid
                else:
                    lo = mid
            return hi

        for st in self.streams.values():
            sp = st.spec
            desc = (sp.height, sp.width)
            x = torch.from_numpy(np.ascontiguousarray(sp.frames[0])).cuda()
            m.forward(x.reshape(-1), [desc], heads=heads)
            k = max(int(sp.n_obj), 1)
            sp.logit_offset = 0.5 * (first_reaching(k, desc) + first_reaching(k + 1, desc))
        torch.cuda.synchronize()

    def _cand_stats(self):
        """Per stream: (objects in its scene, mean candidates per frame)."""
        return {sid: (self.streams[sid].spec.n_obj, round(float(np.mean(c)), 1) if c else None)
                for sid, c in self.cand.items()}

    # ---- producer side -------------------------------------------------------
    def _free_slot(self):
        for i, sl in enumerate(self.slots):
            if not sl["busy"]:
                return i
        return None

    def _launch(self, slot_i, jobs):
        torch = self.torch
        sl = self.slots[slot_i]
        m = sl["m"]
        t0 = time.perf_counter()
        s = sl["stream"]
        heads, dets = sl["heads"], sl["dets"]
        descs, off = [], 0
        offs = sl["off_host"][:len(jobs)]
        offs.numpy()[:] = [self.streams[j.sid].spec.logit_offset for j in jobs]
        with torch.cuda.stream(s):
            for j in jobs:
                st = self.streams[j.sid]
                src = st.pinned[st.spec.frame_index(j.t)]
                n = src.numel()
                sl["dev"][off:off + n].copy_(src, non_blocking=True)
                off += n
                descs.append((st.spec.height, st.spec.width))
            sl["off"][:len(jobs)].copy_(offs, non_blocking=True)
            if sl["graph"] is not None:
                sl["graph"].launch_batch(descs, stream=s)
            else:
                m.forward(sl["dev"][:off], descs, heads=heads, stream=s)
                m.decode(heads, descs, self.conf_thr, self.nms_iou, dets=dets, stream=s, logit_offset=sl["off"])
            ev = torch.cuda.Event()
            ev.record(s)
        sl["busy"] = True
        self.t_launch += time.perf_counter() - t0
        return {"slot": slot_i, "jobs": jobs, "descs": descs, "dets": dets, "heads": heads, "event": ev}

    def run(self, duration, post_queue_depth=4, warmup=0.0):
        """Serve for `duration` seconds of arrivals; returns the statistics dict
        (frames arriving in the first `warmup` seconds are served but not counted)."""
        torch = self.torch
        q = queue.Queue(maxsize=post_queue_depth)
        post = threading.Thread(target=self._post_worker, args=(q,), daemon=True)
        post.start()
        pending = []
        next_t = {sid: 0 for sid in self.streams}
        t_start = time.perf_counter()
        n_batches = 0
        while True:
            now = time.perf_counter() - t_start
            for sid, st in self.streams.items():
                sp = st.spec
                while True:
                    arr = sp.phase + next_t[sid] / sp.fps
                    if arr > now or arr >= duration:
                        break
                    pending.append(FrameJob(sid, next_t[sid], t_start + arr))
                    next_t[sid] += 1
            done_arrivals = all(st.spec.phase + next_t[sid] / st.spec.fps >= duration
                                for sid, st in self.streams.items())
            slot = self._free_slot()
            if pending and slot is not None:
                pending.sort(key=lambda j: j.arrival)
                m = self.slots[slot]["m"]
                want = pending[:self.max_batch]
                descs = [(self.streams[j.sid].spec.height, self.streams[j.sid].spec.width) for j in want]
                with self.lock:
                    k = m.admit(descs, self.in_flight_bytes, self.hbm_budget)
                    batch = want[:k]
                    self.in_flight_bytes += sum(m.frame_bytes(h, w) for h, w in descs[:k])
                if k == 0:
                    self.budget_stalls += 1
                elif k < len(want):
                    self.budget_cut += 1
                if batch:
                    for j in batch:
                        j.admitted = time.perf_counter()
                    pending = pending[len(batch):]
                    q.put(self._launch(slot, batch))
                    n_batches += 1
                    continue
            if done_arrivals and not pending:
                break
            time.sleep(0.0002)
        q.put(None)
        post.join()
        wall = time.perf_counter() - t_start
        counted = [r for r in self.results if r["arrival"] >= t_start + warmup]
        lat = np.array([r["latency"] for r in counted]) * 1e3
        span = wall - warmup
        stats = {"frames": len(counted), "batches": n_batches, "wall_s": wall,
                 "fps": len(counted) / span if span > 0 else 0.0,
                 "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
                 "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
                 "mean_batch": len(self.results) / max(n_batches, 1),
                 "budget_bytes": self.hbm_budget, "budget_stalls": self.budget_stalls,
                 "budget_cut_batches": self.budget_cut,
                 "candidates_per_frame": self._cand_stats(),
                 "host_launch_s": self.t_launch, "host_post_s": self.t_post,
                 "post_parts_s": dict(self.t_parts)}
        return stats

    # ---- post-processing side (the paper's separate post-processing worker) --------
    def _post_worker(self, q):
        torch = self.torch
        while True:
            item = q.get()
            if item is None:
                return
            item["event"].synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(self.post_stream):
                self.post_stream.wait_event(item["event"])
                jobs = sorted(enumerate(item["jobs"]), key=lambda x: (x[1].sid, x[1].t))
                # frames of a stream must be associated in order: the first frame of
                # every stream goes in one batched round, later ones in further rounds
                rounds, seen = [], {}
                for f, j in jobs:
                    r = seen.get(j.sid, 0)
                    seen[j.sid] = r + 1
                    while len(rounds) <= r:
                        rounds.append([])
                    rounds[r].append((f, j))
                m = self.slots[item["slot"]]["m"]
                dets = item["dets"]
                n = len(jobs)
                counts = dets["count"][:n].cpu().numpy()
                ncand = dets["n_cand"][:n].cpu().numpy()
                for f, j in enumerate(item["jobs"]):
                    self.cand[j.sid].append(int(ncand[f]))
                boxes_all = dets["boxes"].view(-1, m.cap, 4)[:n].cpu().numpy()
                i0 = len(self.results)
                assoc = self._associate_round_device if self.device_assoc else self._associate_round
                for rnd in rounds:
                    assoc(sorted(rnd, key=lambda x: x[0]), m, dets, counts, boxes_all)
                done = time.perf_counter()
                for r in self.results[i0:]:
                    r["latency"] = done - r["arrival"]
            self.t_post += time.perf_counter() - t0
            with self.lock:
                self.in_flight_bytes -= sum(m.frame_bytes(h, w) for h, w in item["descs"])
                self.slots[item["slot"]]["busy"] = False

    def _associate_round(self, rnd, m, dets, counts, boxes_all):
        """Appendix A items 4-9 for a set of frames of distinct streams, batched on the device."""
        torch = self.torch
        s = self.post_stream
        cap = m.cap
        dev = self.pool.device
        sts = [self.streams[j.sid] for _, j in rnd]
        counts_t = [len(st.ids) for st in sts]
        tb = np.concatenate([[0], np.cumsum(counts_t)]).astype(np.int32)
        T = int(tb[-1])
        maxd = int(max((counts[f] for f, _ in rnd), default=0))
        tm = self.t_parts
        t0 = time.perf_counter()
        for st in sts:                               # host FP64 predict, in place per stream
            if len(st.ids):
                jde_kf_predict(st.mean, st.cov)
        t1 = time.perf_counter()
        tm["predict"] += t1 - t0
        cost_h = None
        if T and maxd:
            rows = torch.from_numpy(np.concatenate([st.rows for st in sts])).to(dev, non_blocking=True)
            fe = self.pool.index_select(0, rows)
            dmean = torch.from_numpy(np.concatenate([st.mean for st in sts])).to(dev, non_blocking=True)
            dcov = torch.from_numpy(np.concatenate([st.cov for st in sts])).to(dev, non_blocking=True)
            sub = self._sub_dets(dets, [f for f, _ in rnd], cap)
            cost = m.cost_batch(fe, dmean, dcov, tb, sub, CHI2_GATE, stream=s)
            cost_h = cost[:, :maxd].cpu().numpy()
        t2 = time.perf_counter()
        tm["cost"] += t2 - t1
        upd_rows, upd_src, new_rows, new_src = [], [], [], []
        for i, (f, j) in enumerate(rnd):
            st = sts[i]
            boxes = boxes_all[f, :counts[f]]
            D = len(boxes)
            det_ids = np.zeros(D, dtype=np.int64)
            zs = jde_box_to_z(boxes) if D else np.zeros((0, 4))
            matched_t = np.zeros(len(st.ids), dtype=bool)
            matched_d = np.zeros(D, dtype=bool)
            ta = time.perf_counter()
            tc = time.thread_time()
            if counts_t[i] and D:
                pairs, _ = jde_assign(cost_h[tb[i]:tb[i + 1], :D], self.max_cost)
                if len(pairs):
                    t_idx, d_idx = pairs[:, 0], pairs[:, 1]
                    jde_kf_update_n(t_idx, d_idx, st.mean, st.cov, zs)
                    det_ids[d_idx] = st.ids[t_idx]
                    matched_t[t_idx] = True
                    matched_d[d_idx] = True
                    upd_rows.extend(st.rows[t_idx].tolist())
                    upd_src.extend((f * cap + d_idx).tolist())
            tb_ = time.perf_counter()
            tm["assign_update"] += tb_ - ta
            tm["assign_update_cpu"] += time.thread_time() - tc
            tm["frames"] += 1
            st.lost[matched_t] = 0
            st.lost[~matched_t] += 1
            keep = st.lost <= self.max_lost
            st.free_rows.extend(st.rows[~keep].tolist())
            st.mean, st.cov = st.mean[keep], st.cov[keep]
            st.ids, st.lost, st.rows = st.ids[keep], st.lost[keep], st.rows[keep]
            new_d = np.nonzero(~matched_d)[0][:len(st.free_rows)]
            if len(new_d):
                m0, c0 = jde_kf_initiate_n(zs[new_d])
                rws = np.array([st.free_rows.pop() for _ in new_d], dtype=np.int64)
                nid = np.arange(st.next_id, st.next_id + len(new_d))
                st.next_id += len(new_d)
                det_ids[new_d] = nid
                st.mean = np.concatenate([st.mean, m0])
                st.cov = np.concatenate([st.cov, c0])
                st.ids = np.concatenate([st.ids, nid])
                st.lost = np.concatenate([st.lost, np.zeros(len(new_d), dtype=np.int64)])
                st.rows = np.concatenate([st.rows, rws])
                new_rows.extend(rws.tolist())
                new_src.extend((f * cap + new_d).tolist())
            self.results.append({"sid": j.sid, "t": j.t, "boxes": boxes.copy(), "ids": det_ids,
                                 "arrival": j.arrival, "latency": 0.0})
            tm["lifecycle"] += time.perf_counter() - tb_
        t3 = time.perf_counter()
        tm["host_assoc"] += t3 - t2
        emb = dets["emb"]
        if upd_rows:
            pr = torch.from_numpy(np.stack([upd_rows, upd_src], axis=1).astype(np.int32)).to(dev, non_blocking=True)
            jde_track_emb_update(pr, emb, self.pool, 0.9, stream=s)
        if new_rows:
            dst = torch.tensor(new_rows, dtype=torch.int64).to(dev, non_blocking=True)
            src = torch.tensor(new_src, dtype=torch.int64).to(dev, non_blocking=True)
            self.pool.index_copy_(0, dst, emb.index_select(0, src))
        s.synchronize()
        tm["update_sync"] += time.perf_counter() - t3
        tm["tracks"] = max(tm["tracks"], T)

    def _associate_round_device(self, rnd, m, dets, counts, boxes_all):
        """The same round with the Kalman filter and the assignment on the device."""
        torch = self.torch
        s = self.post_stream
        cap = m.cap
        dev = self.pool.device
        sts = [self.streams[j.sid] for _, j in rnd]
        counts_t = [len(st.ids) for st in sts]
        tb = np.concatenate([[0], np.cumsum(counts_t)]).astype(np.int32)
        T = int(tb[-1])
        maxd = int(max((counts[f] for f, _ in rnd), default=0))
        tm = self.t_parts
        t0 = time.perf_counter()
        det_of_track = np.full(T, -1, dtype=np.int32)
        if T:
            rows = torch.from_numpy(np.concatenate([st.rows for st in sts])).to(dev, non_blocking=True)
            dmean = self.kmean.index_select(0, rows)
            dcov = self.kcov.index_select(0, rows)
            jde_kf_predict_dev(dmean, dcov, stream=s)
            if maxd:
                sub = self._sub_dets(dets, [f for f, _ in rnd], cap)
                fe = self.pool.index_select(0, rows)
                cost = m.cost_batch(fe, dmean, dcov, tb, sub, CHI2_GATE, stream=s)
                out = jde_assign_dev(cost, tb, sub, cap, self.max_cost, stream=s)
                jde_kf_update_dev(tb, out["det_of_track"], sub, cap, dmean, dcov, stream=s)
            self.kmean.index_copy_(0, rows, dmean)
            self.kcov.index_copy_(0, rows, dcov)
            if maxd:
                det_of_track = out["det_of_track"][:T].cpu().numpy()
        t2 = time.perf_counter()
        tm["cost"] += t2 - t0
        upd_rows, upd_src, new_rows, new_src = [], [], [], []
        init_rows, init_z = [], []
        for i, (f, j) in enumerate(rnd):
            st = sts[i]
            boxes = boxes_all[f, :counts[f]]
            D = len(boxes)
            dtr = det_of_track[tb[i]:tb[i + 1]]
            matched_t = dtr >= 0
            det_ids = np.zeros(D, dtype=np.int64)
            matched_d = np.zeros(D, dtype=bool)
            det_ids[dtr[matched_t]] = st.ids[matched_t]
            matched_d[dtr[matched_t]] = True
            upd_rows.extend(st.rows[matched_t].tolist())
            upd_src.extend((f * cap + dtr[matched_t]).tolist())
            tm["frames"] += 1
            st.lost[matched_t] = 0
            st.lost[~matched_t] += 1
            keep = st.lost <= self.max_lost
            st.free_rows.extend(st.rows[~keep].tolist())
            st.ids, st.lost, st.rows = st.ids[keep], st.lost[keep], st.rows[keep]
            new_d = np.nonzero(~matched_d)[0][:len(st.free_rows)]
            if len(new_d):
                rws = np.array([st.free_rows.pop() for _ in new_d], dtype=np.int64)
                nid = np.arange(st.next_id, st.next_id + len(new_d))
                st.next_id += len(new_d)
                det_ids[new_d] = nid
                st.ids = np.concatenate([st.ids, nid])
                st.lost = np.concatenate([st.lost, np.zeros(len(new_d), dtype=np.int64)])
                st.rows = np.concatenate([st.rows, rws])
                new_rows.extend(rws.tolist())
                new_src.extend((f * cap + new_d).tolist())
                init_rows.append(rws)
                init_z.append(jde_box_to_z(boxes[new_d]))
            self.results.append({"sid": j.sid, "t": j.t, "boxes": boxes.copy(), "ids": det_ids,
                                 "arrival": j.arrival, "latency": 0.0})
        t3 = time.perf_counter()
        tm["host_assoc"] += t3 - t2
        emb = dets["emb"]
        if upd_rows:
            pr = torch.from_numpy(np.stack([upd_rows, upd_src], axis=1).astype(np.int32)).to(dev, non_blocking=True)
            jde_track_emb_update(pr, emb, self.pool, 0.9, stream=s)
        if new_rows:
            dst = torch.tensor(new_rows, dtype=torch.int64).to(dev, non_blocking=True)
            src = torch.tensor(new_src, dtype=torch.int64).to(dev, non_blocking=True)
            self.pool.index_copy_(0, dst, emb.index_select(0, src))
            m0, c0 = jde_kf_initiate_n(np.concatenate(init_z))
            self.kmean.index_copy_(0, dst, torch.from_numpy(m0).to(dev, non_blocking=True))
            self.kcov.index_copy_(0, dst, torch.from_numpy(c0).to(dev, non_blocking=True))
        s.synchronize()
        tm["update_sync"] += time.perf_counter() - t3
        tm["tracks"] = max(tm["tracks"], T)

    @staticmethod
    def _sub_dets(dets, frames, cap):
        """Views of the detection buffers restricted to the given frames, in order
        (a contiguous selection when the frames are consecutive, else a gather)."""
        idx = np.asarray(frames)
        if np.all(np.diff(idx) == 1):
            lo, hi = int(idx[0]), int(idx[-1]) + 1
            return {k: (v[lo:hi] if k in ("count", "n_cand", "overflow") else
                        v.view(-1, cap, *v.shape[1:])[lo:hi].reshape(-1, *v.shape[1:]))
                    for k, v in dets.items()}
        import torch
        ti = torch.from_numpy(idx).to(dets["count"].device)
        return {k: (v.index_select(0, ti) if k in ("count", "n_cand", "overflow") else
                    v.view(-1, cap, *v.shape[1:]).index_select(0, ti).reshape(-1, *v.shape[1:]).contiguous())
                for k, v in dets.items()}


def synthetic_streams(n_streams, seed, frames_per_stream=4, fps=30.0, resolutions=((608, 1088), (480, 864),
                      (320, 576)), objects=(20, 200)):
    """Seeded stream specs: resolution uniform over `resolutions`, 20-200 objects,
    random phase, frames_per_stream consecutive frames of a moving scene (the
    confidence offset for the stream's density is set by Server.calibrate_density)."""
    from jde_inputs import scene_batch
    rng = np.random.Generator(np.random.PCG64([seed, 23]))
    out = []
    for s in range(n_streams):
        h, w = resolutions[int(rng.integers(len(resolutions)))]
        n_obj = int(rng.integers(objects[0], objects[1] + 1))
        fr = scene_batch(seed, frames_per_stream, h, w, n_obj=n_obj, stream=s)
        out.append(StreamSpec(s, h, w, fps, float(rng.uniform(0, 1.0 / fps)), fr, 0.0, n_obj))
    return out
