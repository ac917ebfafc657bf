"""Benchmark of the JDE hot path on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic
3x608x1088 frames already resident in HBM: the JDE forward (Darknet-53, FPN,
three heads), decode + confidence threshold, sort, NMS, embedding
L2-normalisation, and the tracks x detections cost matrix (cosine distance with
Mahalanobis gating) of every frame against 40 synthetic tracks.

Prints ONE JSON line on stdout; a per-launch breakdown goes to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--precision bf16]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frames/s at 1088x608 (BF16 batched vs FP32 batch-1) + p99 frame latency"
PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3, "fp8": 5000.0}
N_TRACKS = 40
K_CAND = 40
CONF, NMS_IOU = 0.5, 0.4


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "conv_bf16_b16_608x1088_traffic.json")


def conv_source_hash(key, tiles):
    """Identifies the conv kernels' source and this workload's tile choice."""
    import hashlib
    h = hashlib.sha256()
    for f in ("conv.hip", "jde_internal.h"):
        with open(os.path.join(ROOT, "paper_2011_03910_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(json.dumps([key, tiles]).encode())
    return h.hexdigest()


def measured_traffic(key, tiles):
    """HBM bytes per conv launch from the committed hardware-counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's counts), or None when
    that summary was taken on other kernel source or another tile choice."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    if rec.get("workload") != key or rec.get("source_sha256") != conv_source_hash(key, tiles):
        return None
    return rec["bytes_per_launch"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(batch, torch):
    """Frames [B, 3, 608, 1088] and, per frame, its own set of N_TRACKS tracks."""
    import numpy as np
    from jde_inputs import FULL, scene_batch, synthetic_dets_tracks
    fr = scene_batch(FULL.seed, batch, FULL.height, FULL.width)
    trk = [synthetic_dets_tracks(FULL.seed + f, N_TRACKS, N_TRACKS, FULL.emb_dim) for f in range(batch)]
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cat = lambda k: cu(np.concatenate([t[k] for t in trk]))
    return cu(fr), cat("trk_emb"), cat("mean"), cat("cov")


class Pipeline:
    """Preallocated buffers and one step of the hot path for a fixed batch."""

    def __init__(self, precision, batch, layers, torch, tune_frames=None, tiles=None, calib_frames=None):
        from jde_inputs import FULL, anchors_px
        from paper_2011_03910_amd import JDE
        self.torch = torch
        self.batch = batch
        self.descs = [(FULL.height, FULL.width)] * batch
        self.m = JDE(FULL.c0, FULL.blocks, FULL.emb_dim, anchors_px(FULL), precision, batch, FULL.height,
                     FULL.width, 512)
        self.m.load_weights(layers)
        self.heads = self.m.head_buffers(self.descs)
        self.dets = self.m.dets_buffers(batch)
        self.track_begin = [N_TRACKS * f for f in range(batch + 1)]
        self.cost = torch.empty((batch * N_TRACKS, self.m.cap), dtype=torch.float32, device="cuda")
        self.tiles = None
        if precision == "fp8":
            # static activation scales from one BF16 pass over this batch
            self.m.calibrate(tune_frames if tune_frames is not None else calib_frames, self.descs, heads=self.heads)
        if tiles is not None:
            self.m.set_tiles(tiles)
            self.tiles = self.m.tiles()
        elif tune_frames is not None:
            t0 = time.perf_counter()
            self.tiles = self.m.autotune(tune_frames, self.descs, heads=self.heads, reps=3)
            log(f"autotuned {precision} b{batch} tiles in {time.perf_counter() - t0:.1f} s: {self.tiles.tolist()}")

    def step(self, frames, trk_emb, mean, cov):
        self.m.forward(frames, self.descs, heads=self.heads)
        self.m.decode(self.heads, self.descs, CONF, NMS_IOU, dets=self.dets)
        self.m.cost_batch(trk_emb, mean, cov, self.track_begin, self.dets, cost=self.cost)

    def capture(self, frames, trk_emb, mean, cov):
        """The same step captured once as a HIP graph (replayed per step)."""
        s = self.torch.cuda.Stream()
        self.graph = self.m.graph_capture(frames, self.descs, self.heads, self.dets, CONF, NMS_IOU,
                                          tracks=(trk_emb, mean, cov, self.track_begin), cost=self.cost, stream=s)
        self.torch.cuda.synchronize()


def run(pipe, inputs, steps, warmup, torch, profile=False, graph=False):
    stream = torch.cuda.current_stream()
    one = (lambda: pipe.graph.launch(stream)) if graph else (lambda: pipe.step(*inputs))
    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    if profile:
        pipe.m.profile_begin(True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record(stream)
        one()
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = sorted(a.elapsed_time(b) for a, b in evs)
    prof = pipe.m.profile_collect() if profile else None
    if profile:
        pipe.m.profile_begin(False)
    return wall, step_ms, prof


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def serve_bench(layers, precision, seconds, tiles, torch):
    """16 synthetic streams at 30 FPS (mixed resolutions, 20-200 objects) through the
    continuous-batching server; per-frame latency = arrival -> tracks updated."""
    from jde_inputs import FULL, anchors_px
    from paper_2011_03910_amd.serve import Server, synthetic_streams
    streams = synthetic_streams(16, FULL.seed, frames_per_stream=2)
    srv = Server(FULL, anchors_px(FULL), layers, streams, precision=precision, max_batch=16, tiles=tiles)
    stats = srv.run(seconds + 0.5, warmup=0.5)
    res = sorted({(s.height, s.width) for s in streams})
    stats.update({"streams": 16, "offered_fps": 16 * 30, "resolutions": [f"{w}x{h}" for h, w in res],
                  "hbm_budget_gb": round(srv.hbm_budget / 1e9, 2)})
    return stats


def cpu_baseline(layers):
    """The FP64 oracle on a bounded sample: one full-resolution frame through
    forward, decode, NMS, normalisation and the cost against 40 tracks."""
    import numpy as np
    from jde_inputs import FULL, scene_batch, synthetic_dets_tracks, anchors_px
    from oracle.network import forward
    from oracle.post import detections
    from oracle.track import cost_matrix
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    fr = scene_batch(FULL.seed, 1, FULL.height, FULL.width)
    trk = synthetic_dets_tracks(FULL.seed, N_TRACKS, N_TRACKS, FULL.emb_dim)
    t0 = time.perf_counter()
    out = forward(fr, layers, FULL.blocks)
    d = detections(out, anchors_px(FULL), CONF, NMS_IOU)
    cost_matrix(trk["trk_emb"], trk["mean"], trk["cov"], d["boxes"], d["emb"])
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "frames/s", "cores": int(cores), "kind": "oracle",
            "sample": f"1 frame 3x608x1088, FP64 numpy: forward + decode + NMS + normalise + "
                      f"{N_TRACKS}-track cost ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp16", "fp32", "fp8"])
    ap.add_argument("--fp32-steps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 batch-1 plain form")
    ap.add_argument("--no-tune", action="store_true", help="built-in tile choice instead of the autotuner")
    ap.add_argument("--serve-seconds", type=float, default=4.0, help="serving run length (0: skip)")
    ap.add_argument("--save-tiles", help="write the tile choices to this JSON file")
    ap.add_argument("--load-tiles", help="use tile choices from this JSON file instead of tuning")
    ap.add_argument("--retune", action="store_true", help="run the autotuner instead of the stored tile choices")
    ap.add_argument("--eager", action="store_true",
                    help="time eager launches instead of replaying the step as a captured HIP graph")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run one plain elementwise copy of this many MiB (FP32 negate, read N + write N "
                         "bytes): the reference dispatch that scales hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (frames are independent, "
              "so more GPUs would each run this same single-GPU path on their own streams)", file=sys.stderr)
        sys.exit(2)

    import torch
    from jde_inputs import FULL, model_weights
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"device: {torch.cuda.get_device_name(0)}")
    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mb} MiB read + {args.copy_probe_mb} MiB written")
        del src, dst
    layers = model_weights(FULL, K_CAND)
    inputs_b = make_inputs(args.batch, torch)

    cache = os.path.join(ROOT, "paper_2011_03910_amd", "tiles_mi355x.json")
    if args.load_tiles:
        saved = json.load(open(args.load_tiles))
    elif not args.retune and not args.no_tune and os.path.exists(cache):
        saved = json.load(open(cache))          # autotuner results for this workload
    else:
        saved = {}
    key = f"{args.precision}_b{args.batch}"
    pipe = Pipeline(args.precision, args.batch, layers, torch, None if args.no_tune else inputs_b[0],
                    saved.get(key), calib_frames=inputs_b[0])
    tiles_out = {key: None if pipe.tiles is None else pipe.tiles.tolist()}
    traffic = measured_traffic(key, tiles_out[key])
    # Throughput and latency from a timed pass with no per-launch events; the
    # per-launch durations (roofline) from a second timed pass of the same steps in
    # which the library brackets every launch with a HIP event pair.
    if not args.eager:
        pipe.capture(*inputs_b)
    wall, step_ms, _ = run(pipe, inputs_b, args.steps, args.warmup, torch, graph=not args.eager)
    wall_p, step_ms_p, prof = run(pipe, inputs_b, args.steps, 1, torch, profile=True)
    log(f"{'graph replay' if not args.eager else 'eager'}: {1e3 * wall / args.steps:.3f} ms/step; eager with "
        f"per-launch events: {1e3 * wall_p / args.steps:.3f} ms/step")
    fps = args.batch * args.steps / wall
    counts = pipe.dets["count"].cpu().numpy()
    ncand = pipe.dets["n_cand"].cpu().numpy()
    log(f"{args.precision} b{args.batch}: {fps:.1f} frames/s, step p50 {pct(step_ms, 50):.2f} ms "
        f"p99 {pct(step_ms, 99):.2f} ms; candidates/frame {ncand.mean():.1f}, kept {counts.mean():.1f}")

    ms, fl, kind, nfwd = prof
    conv = (kind == 1) | (kind == 6)  # implicit-GEMM and persistent pointwise conv launches
    conv_ms = ms[conv].sum() / nfwd
    conv_flop = fl[conv].sum()
    n_launch = int(conv.sum())
    achieved = conv_flop / (conv_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    fwd_ms = ms.sum() / nfwd
    log(f"forward launches: {len(ms)}; conv {n_launch} launches {conv_ms:.3f} ms/step "
        f"({conv_flop / 1e9:.1f} GFLOP) -> {achieved:.1f} TFLOP/s; all forward launches {fwd_ms:.3f} ms")
    if (kind == 2).any():
        # stem fused with the first downsample conv: HBM-bound (FP32 frames in, the
        # stride-2 level's 64 channels out)
        t2 = ms[kind == 2].sum() / nfwd
        nbytes = args.batch * (3 * 608 * 1088 * 4 + 304 * 544 * 64 * (4 if args.precision == "fp32" else 2))
        log(f"fused stem + downsample: {t2 * 1e3:.1f} us, {nbytes / 1e6:.0f} MB algorithmic -> "
            f"{nbytes / (t2 * 1e-3) / 1e12:.2f} TB/s of 8")
    for i in range(len(ms)):
        t = ms[i] / nfwd
        log(f"  op {i:2d} kind {kind[i]} {t * 1e3:9.1f} us  {fl[i] / 1e9:8.2f} GFLOP  "
            f"{(fl[i] / (t * 1e-3) / 1e12 if t > 0 else 0):7.1f} TFLOP/s")
    del pipe
    torch.cuda.empty_cache()

    fp32 = None
    if not args.no_fp32:
        in1 = (inputs_b[0][:1].contiguous(), inputs_b[1][:N_TRACKS], inputs_b[2][:N_TRACKS], inputs_b[3][:N_TRACKS])
        p32 = Pipeline("fp32", 1, layers, torch, None if args.no_tune else in1[0], saved.get("fp32_b1"))
        tiles_out["fp32_b1"] = None if p32.tiles is None else p32.tiles.tolist()
        w32, s32, _ = run(p32, in1, args.fp32_steps, 3, torch)
        fp32 = {"fps": 1 * args.fp32_steps / w32, "p50_ms": pct(s32, 50), "p99_ms": pct(s32, 99)}
        log(f"fp32 b1: {fp32['fps']:.1f} frames/s, p50 {fp32['p50_ms']:.2f} ms")
        del p32
        torch.cuda.empty_cache()

    if args.save_tiles:
        json.dump(tiles_out, open(args.save_tiles, "w"))
    serving = None
    if args.serve_seconds > 0:
        serving = serve_bench(layers, args.precision, args.serve_seconds, tiles_out.get(key), torch)
        log(f"serving: {serving}")
        torch.cuda.empty_cache()
    cpu = None if args.no_cpu else cpu_baseline(layers)
    if cpu:
        log(f"cpu oracle: {cpu['value']:.4f} frames/s on {cpu['cores']} threads")

    rec = {
        "metric": METRIC, "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"JDE Darknet-53+FPN+3 heads (E=512), 3x608x1088 synthetic scene frames, "
                               f"{args.precision.upper()} batch {args.batch}, ~{K_CAND} candidates/frame; "
                               f"forward + decode + NMS + L2-normalise + {N_TRACKS}-track gated cost",
                   "global_batch": args.batch, "seq_len": None, "parallelism": "none (1 GPU)",
                   "resolution": "608x1088"},
        "p50_frame_latency_ms": round(pct(step_ms, 50), 3), "p99_frame_latency_ms": round(pct(step_ms, 99), 3),
        "fp32_b1": None if fp32 is None else {k: round(v, 3) for k, v in fp32.items()},
        "speedup_vs_fp32_b1": None if fp32 is None else round(fps / fp32["fps"], 2),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": traffic,
                     "kernel": f"conv launches conv_dma/conv_igemm/conv_pw_stream ({n_launch} launches/step, {conv_flop / 1e9:.1f} GFLOP/step, "
                               f"mean {conv_ms / n_launch * 1e3:.1f} us/launch)"},
        "serving": None if serving is None else {k: (round(v, 3) if isinstance(v, float) else v)
                                                  for k, v in serving.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
