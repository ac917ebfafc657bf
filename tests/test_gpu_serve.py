"""GPU test of the serving loop: continuous batching over concurrent streams.

Each stream's per-frame results (detections after NMS and the track id given
to each detection) are the same when the stream is served alone and when it
shares ragged batches with other streams of other resolutions.
"""

import sys

import numpy as np
import pytest

from jde_inputs import TINY, tiny_frame
from tests.helpers import weights, anchors

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _streams(sids):
    from paper_2011_03910_amd.serve import StreamSpec
    sizes = {0: (192, 320), 1: (128, 224), 2: (96, 160), 3: (192, 320)}
    out = []
    for s in sids:
        h, w = sizes[s]
        fr = np.stack([tiny_frame(TINY.seed, 100 * s + k, h, w) for k in range(3)])
        out.append(StreamSpec(s, h, w, 60.0, 0.004 * s, fr))
    return out


def _serve(sids, duration=0.4):
    from paper_2011_03910_amd.serve import Server
    srv = Server(TINY, anchors("tiny"), weights("tiny", 50), _streams(sids), precision="fp32", max_batch=4,
                 max_tracks=128, cap=256)
    stats = srv.run(duration)
    by = {}
    for r in srv.results:
        by[(r["sid"], r["t"])] = r
    return stats, by


def test_stream_results_same_alone_and_in_mix():
    import torch
    assert torch.cuda.is_available()
    _say("case: serve mix of 4 streams")
    st_mix, mix = _serve([0, 1, 2, 3])
    _say(f"  mix: {st_mix}")
    assert st_mix["frames"] >= 4 * 20 and st_mix["mean_batch"] > 1.0
    for sid in (1, 3):
        _say(f"case: serve stream {sid} alone")
        st_one, one = _serve([sid])
        keys = sorted(k for k in one if k[0] == sid)
        assert len(keys) >= 20
        for k in keys:
            a, b = one[k], mix[k]
            assert a["boxes"].shape == b["boxes"].shape, k
            np.testing.assert_allclose(a["boxes"], b["boxes"], rtol=1e-5, atol=1e-3)
            np.testing.assert_array_equal(a["ids"], b["ids"])
        _say(f"  stream {sid}: {len(keys)} frames identical alone and in the mix; "
             f"tracks {max(int(x['ids'].max(initial=0)) for x in one.values())}")
