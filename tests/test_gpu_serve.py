"""GPU test of the serving loop: continuous batching over concurrent streams.

Each stream's per-frame results (detections after NMS and the track id given
to each detection) are the same when the stream is served alone and when it
shares ragged batches with other streams of other resolutions and densities
(each stream has its own confidence offset), under a device-memory budget that
holds only two frames at a time, in FP32 and in BF16.
"""

import sys

import numpy as np
import pytest

from jde_inputs import TINY, tiny_frame
from tests.helpers import weights, anchors

pytestmark = pytest.mark.gpu

SIZES = {0: (192, 320), 1: (128, 224), 2: (96, 160), 3: (192, 320)}
OFFSETS = {0: 0.0, 1: 0.8, 2: -0.5, 3: 1.5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _streams(sids):
    from paper_2011_03910_amd.serve import StreamSpec
    out = []
    for s in sids:
        h, w = SIZES[s]
        fr = np.stack([tiny_frame(TINY.seed, 100 * s + k, h, w) for k in range(3)])
        # streams 0, 1 and 3 arrive together: three frames that a budget of two
        # 192x320 frames cannot admit at once
        out.append(StreamSpec(s, h, w, 60.0, 0.008 if s == 2 else 0.0, fr, OFFSETS[s], 0))
    return out


def _serve(sids, precision, duration=0.4, budget_frames=None, device_assoc=True):
    from paper_2011_03910_amd.serve import Server
    srv = Server(TINY, anchors("tiny"), weights("tiny", 50), _streams(sids), precision=precision, max_batch=4,
                 max_tracks=128, cap=256, device_assoc=device_assoc)
    if budget_frames is not None:
        srv.hbm_budget = budget_frames * srv.slots[0]["m"].frame_bytes(192, 320)
    stats = srv.run(duration)
    by = {}
    for r in srv.results:
        by[(r["sid"], r["t"])] = r
    return stats, by


@pytest.mark.parametrize("precision,device_assoc", [("fp32", False), ("fp32", True), ("bf16", True)])
def test_stream_results_same_alone_and_in_mix(precision, device_assoc):
    import torch
    assert torch.cuda.is_available()
    _say(f"case: serve mix of 4 streams ({precision}, device association {device_assoc}, budget of two 192x320 "
         f"frames)")
    st_mix, mix = _serve([0, 1, 2, 3], precision, budget_frames=2, device_assoc=device_assoc)
    _say(f"  mix: {st_mix}")
    assert st_mix["frames"] >= 4 * 20 and st_mix["mean_batch"] > 1.0
    assert st_mix["budget_stalls"] + st_mix["budget_cut_batches"] > 0
    for sid in (1, 3):
        _say(f"case: serve stream {sid} alone ({precision})")
        st_one, one = _serve([sid], precision, device_assoc=device_assoc)
        keys = sorted(k for k in one if k[0] == sid)
        assert len(keys) >= 20
        for k in keys:
            a, b = one[k], mix[k]
            assert a["boxes"].shape == b["boxes"].shape, k
            np.testing.assert_allclose(a["boxes"], b["boxes"], rtol=1e-5, atol=1e-3)
            np.testing.assert_array_equal(a["ids"], b["ids"])
        _say(f"  stream {sid}: {len(keys)} frames identical alone and in the mix; "
             f"tracks {max(int(x['ids'].max(initial=0)) for x in one.values())}")


def test_device_association_equals_host_association():
    """The serving loop gives the same detections and track ids with the Kalman
    filter and the assignment on the device as on the host (the device kernels
    take the host code's FP64 steps)."""
    import torch
    assert torch.cuda.is_available()
    _say("case: serve mix, device vs host association")
    _, dev = _serve([0, 1, 2, 3], "fp32", device_assoc=True)
    _, host = _serve([0, 1, 2, 3], "fp32", device_assoc=False)
    keys = sorted(set(dev) & set(host))
    assert len(keys) >= 80
    for k in keys:
        np.testing.assert_array_equal(dev[k]["boxes"], host[k]["boxes"])
        np.testing.assert_array_equal(dev[k]["ids"], host[k]["ids"])
    _say(f"  {len(keys)} frames: identical boxes and ids; tracks up to "
         f"{max(int(x['ids'].max(initial=0)) for x in dev.values())}")


def test_serving_with_graph_replays_equals_eager_launches():
    """Full network, BF16: the serving loop replaying each slot's any-batch graph
    gives the same detections and ids as launching forward + decode eagerly."""
    import torch
    from jde_inputs import FULL, scene_batch
    from paper_2011_03910_amd.serve import Server, StreamSpec
    assert torch.cuda.is_available()
    _say("case: serve full bf16, graph replays vs eager launches")
    sizes = {0: (320, 576), 1: (480, 864), 2: (320, 576)}

    def run(use_graph):
        streams = [StreamSpec(s, h, w, 30.0, 0.0 if s < 2 else 0.01, scene_batch(FULL.seed, 3, h, w, stream=s),
                              0.3 * s, 0) for s, (h, w) in sizes.items()]
        srv = Server(FULL, anchors("full"), weights("full", 100), streams, precision="bf16", max_batch=3,
                     max_tracks=256, cap=512, use_graph=use_graph)
        assert (srv.slots[0]["graph"] is not None) == use_graph
        srv.run(0.5)
        return {(r["sid"], r["t"]): r for r in srv.results}

    g, e = run(True), run(False)
    keys = sorted(set(g) & set(e))
    assert len(keys) >= 30
    for k in keys:
        np.testing.assert_array_equal(g[k]["boxes"], e[k]["boxes"])
        np.testing.assert_array_equal(g[k]["ids"], e[k]["ids"])
    _say(f"  {len(keys)} frames identical, {sum(len(g[k]['ids']) for k in keys)} detections")
