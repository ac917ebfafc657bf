"""Seeded mixes of frame sizes for uneven (ragged) batches.

The paper batches frames for inference (Sec. 4.2); a serving batch can hold
frames of several video streams at different resolutions.  A mix draws the
proportions of 608x1088, 480x864 and 320x576 frames from Dirichlet(1, 1, 1)
and the counts of a batch of `total` frames from the multinomial with those
proportions, then shuffles the order.  A pure function of (seed, total).
"""

from functools import lru_cache

import numpy as np

MIX_SIZES = ((608, 1088), (480, 864), (320, 576))


def ragged_mix(seed: int, total: int, sizes=MIX_SIZES):
    """List of `total` (h, w) frame sizes."""
    r = np.random.Generator(np.random.PCG64([seed, 29, total]))
    p = r.dirichlet(np.ones(len(sizes)))
    counts = r.multinomial(total, p)
    out = [sizes[i] for i, c in enumerate(counts) for _ in range(int(c))]
    order = r.permutation(total)
    return [out[i] for i in order]


@lru_cache(maxsize=64)
def _pool_frame(seed, stream, t, h, w):
    from .frames import scene_frame
    f = scene_frame(seed, stream, t, h, w).ravel()
    f.setflags(write=False)
    return f


def mix_frames(seed: int, sizes, stream_base: int = 200, pool: int = 8):
    """FP32 frames for a list of sizes, packed back to back (frame k: 3*h*w
    floats).  Each resolution i of MIX_SIZES has its own moving scene (synthetic
    stream stream_base + i); the k-th frame of a mix is frame k mod `pool` of the
    scene of its size, so mixes of any length render at most `pool` frames per
    resolution."""
    return np.concatenate([_pool_frame(seed, stream_base + MIX_SIZES.index((h, w)), k % pool, h, w)
                           for k, (h, w) in enumerate(sizes)])
