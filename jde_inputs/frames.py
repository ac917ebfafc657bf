"""Seeded synthetic frames.

* ``tiny_frame``: pixels i.i.d. U[0, 1], shape [3, H, W] FP32.
* ``scene_frame``: a stand-in for a FullHD pedestrian sequence resized to
  1088x608 (the paper's MOT16 inputs, Sec. 5): a static smooth value-noise
  background (4 octaves, cells 64/32/16/8 px, amplitudes 1, 1/2, 1/4, 1/8,
  bilinearly interpolated, normalised to [0, 1]) and tall textured rectangles
  (height U[40, 300] px at 608 rows, aspect w/h U[0.3, 0.6]) moving at constant
  velocity U[-4, 4]^2 px/frame and bouncing off the borders.  Each rectangle has
  a two-colour stripe or checker texture with period U[4, 16] px.  Objects are
  drawn in index order.  Sizes and speeds scale with H / 608.

Frame t of stream s is a pure function of (seed, s, t).  No MOT16 content is
reproduced.
"""

from functools import lru_cache

import numpy as np

_OCTAVES = ((64, 1.0), (32, 0.5), (16, 0.25), (8, 0.125))


def _rng(*key):
    return np.random.Generator(np.random.PCG64(list(key)))


def tiny_frame(seed: int, index: int = 0, height: int = 192, width: int = 320) -> np.ndarray:
    """[3, H, W] FP32 pixels i.i.d. uniform on [0, 1)."""
    r = _rng(seed, 7, index)
    return r.random((3, height, width)).astype(np.float32)


@lru_cache(maxsize=8)
def _background(seed, stream, height, width):
    bg = _value_noise(_rng(seed, 13, stream), height, width)
    bg.setflags(write=False)
    return bg


def _value_noise(r, height, width):
    out = np.zeros((3, height, width))
    ys = np.arange(height) + 0.5
    xs = np.arange(width) + 0.5
    for cell, amp in _OCTAVES:
        gh = height // cell + 2
        gw = width // cell + 2
        g = r.random((3, gh, gw))
        gy = ys / cell
        gx = xs / cell
        y0 = np.floor(gy).astype(np.int64)
        x0 = np.floor(gx).astype(np.int64)
        fy = (gy - y0)[:, None]
        fx = (gx - x0)[None, :]
        a = g[:, y0][:, :, x0]
        b = g[:, y0][:, :, x0 + 1]
        c = g[:, y0 + 1][:, :, x0]
        d = g[:, y0 + 1][:, :, x0 + 1]
        out += amp * ((a * (1 - fx) + b * fx) * (1 - fy) + (c * (1 - fx) + d * fx) * fy)
    lo = out.min()
    hi = out.max()
    return (out - lo) / (hi - lo)


def scene_objects(seed: int, stream: int, n_obj: int, height: int, width: int):
    """Per-object parameters of one stream: a list of dicts."""
    r = _rng(seed, 11, stream)
    sc = height / 608.0
    objs = []
    for _ in range(n_obj):
        h = r.uniform(40.0, 300.0) * sc
        w = h * r.uniform(0.3, 0.6)
        objs.append(dict(
            w=w, h=h,
            x0=r.uniform(0.0, width - w), y0=r.uniform(0.0, height - h),
            vx=r.uniform(-4.0, 4.0) * sc, vy=r.uniform(-4.0, 4.0) * sc,
            period=r.uniform(4.0, 16.0) * sc,
            checker=bool(r.random() < 0.5),
            col0=r.random(3), col1=r.random(3),
        ))
    return objs


def _bounce(p0, v, t, span):
    """Position after t steps of constant velocity, reflected inside [0, span]."""
    if span <= 0:
        return 0.0
    u = np.mod(p0 + v * t, 2.0 * span)
    return u if u <= span else 2.0 * span - u


def object_box(obj, t, height, width):
    """(x1, y1, x2, y2) of an object at frame t, in pixels."""
    x = _bounce(obj["x0"], obj["vx"], t, width - obj["w"])
    y = _bounce(obj["y0"], obj["vy"], t, height - obj["h"])
    return x, y, x + obj["w"], y + obj["h"]


def scene_frame(seed: int, stream: int, t: int, height: int = 608, width: int = 1088,
                n_obj: int = 40) -> np.ndarray:
    """[3, H, W] FP32 frame t of synthetic stream ``stream``."""
    img = _background(seed, stream, height, width).copy()
    for obj in scene_objects(seed, stream, n_obj, height, width):
        x1, y1, x2, y2 = object_box(obj, t, height, width)
        ix1, iy1 = int(np.floor(x1)), int(np.floor(y1))
        ix2, iy2 = min(int(np.ceil(x2)), width), min(int(np.ceil(y2)), height)
        if ix2 <= ix1 or iy2 <= iy1:
            continue
        yy = (np.arange(iy1, iy2) - y1)[:, None]
        xx = (np.arange(ix1, ix2) - x1)[None, :]
        half = obj["period"] / 2.0
        band = np.floor(xx / half).astype(np.int64)
        if obj["checker"]:
            band = band + np.floor(yy / half).astype(np.int64)
        else:
            band = np.broadcast_to(band, (iy2 - iy1, ix2 - ix1))
        sel = (band % 2 == 0)
        for c in range(3):
            img[c, iy1:iy2, ix1:ix2] = np.where(sel, obj["col0"][c], obj["col1"][c])
    return img.astype(np.float32)


def scene_batch(seed: int, n: int, height: int = 608, width: int = 1088, n_obj: int = 40,
                stream: int = 0, t0: int = 0) -> np.ndarray:
    """[n, 3, H, W] FP32: frames t0 .. t0+n-1 of one stream."""
    return np.stack([scene_frame(seed, stream, t0 + i, height, width, n_obj) for i in range(n)])


def capture_frame(seed: int, stream: int, t: int, height: int = 1080, width: int = 1920,
                  n_obj: int = 40) -> np.ndarray:
    """[H, W, 3] uint8 RGB frame t of a synthetic stream as a capture device
    delivers it (FullHD by default): the scene of ``scene_frame`` at that size,
    quantised to 8 bits."""
    f = scene_frame(seed, stream, t, height, width, n_obj)
    return np.ascontiguousarray(np.clip(np.rint(f * 255.0), 0, 255).astype(np.uint8).transpose(1, 2, 0))
