"""FP64 oracle of frame ingest (test infrastructure only).

The paper's pipeline captures FullHD video (Sec. 4.4: a capture process feeds
the model) and runs the model on frames resized to 1088x608 (Sec. 5.1).  The
resize method is not stated; the reading used here (and by the product):

* source: 8-bit RGB pixels, row-major [H_in, W_in, 3];
* letterbox: scale r = min(h / H_in, w / W_in) keeps the aspect ratio, the
  resized image is round(W_in r) x round(H_in r) pixels (nearest integer,
  halves rounded up), placed at column
  floor((w - new_w) / 2) and row floor((h - new_h) / 2); the border is 0.5;
* bilinear resampling with pixel centres aligned: output pixel u of the resized
  image samples the source at s = (u + 1/2) (W_in / new_w) - 1/2, clamped to
  [0, W_in - 1], interpolating between floor(s) and floor(s) + 1 (clamped);
* value / 255, output [3, h, w] (the model's NCHW input in [0, 1]).
"""

import math

import numpy as np

PAD = 0.5


def letterbox_geometry(src_h, src_w, h, w):
    """(new_h, new_w, top, left) of the resized image inside the h x w frame."""
    r = min(h / src_h, w / src_w)
    new_w = int(math.floor(src_w * r + 0.5))        # nearest, halves up
    new_h = int(math.floor(src_h * r + 0.5))
    new_w = max(min(new_w, w), 1)
    new_h = max(min(new_h, h), 1)
    return new_h, new_w, (h - new_h) // 2, (w - new_w) // 2


def _axis(n_out, n_in):
    """Source indices (i0, i1) and weight of i1 for each output coordinate."""
    s = (np.arange(n_out) + 0.5) * (n_in / n_out) - 0.5
    s = np.clip(s, 0.0, n_in - 1)
    i0 = np.floor(s).astype(np.int64)
    i1 = np.minimum(i0 + 1, n_in - 1)
    return i0, i1, s - i0


def resize_bilinear(img, new_h, new_w):
    """img [H, W, C] (any numeric) -> [new_h, new_w, C] FP64, bilinear as above."""
    img = np.asarray(img, dtype=np.float64)
    y0, y1, fy = _axis(new_h, img.shape[0])
    x0, x1, fx = _axis(new_w, img.shape[1])
    fy = fy[:, None, None]
    fx = fx[None, :, None]
    top = img[y0][:, x0] * (1 - fx) + img[y0][:, x1] * fx
    bot = img[y1][:, x0] * (1 - fx) + img[y1][:, x1] * fx
    return top * (1 - fy) + bot * fy


def ingest(frame_u8, h, w):
    """One 8-bit RGB frame [H_in, W_in, 3] -> the model input [3, h, w] FP64 in [0, 1]."""
    src_h, src_w = frame_u8.shape[:2]
    new_h, new_w, top, left = letterbox_geometry(src_h, src_w, h, w)
    out = np.full((h, w, 3), PAD)
    out[top:top + new_h, left:left + new_w] = resize_bilinear(frame_u8, new_h, new_w) / 255.0
    return np.ascontiguousarray(out.transpose(2, 0, 1))


def ingest_pixel(frame_u8, h, w, c, y, x):
    """The same value for one output pixel, by a direct scalar evaluation (used to
    pin the vectorised form)."""
    src_h, src_w = frame_u8.shape[:2]
    new_h, new_w, top, left = letterbox_geometry(src_h, src_w, h, w)
    u, v = x - left, y - top
    if not (0 <= u < new_w and 0 <= v < new_h):
        return PAD

    def coord(t, n_out, n_in):
        s = min(max((t + 0.5) * (n_in / n_out) - 0.5, 0.0), n_in - 1)
        i0 = int(math.floor(s))
        return i0, min(i0 + 1, n_in - 1), s - i0

    ya, yb, wy = coord(v, new_h, src_h)
    xa, xb, wx = coord(u, new_w, src_w)
    p = lambda yy, xx: float(frame_u8[yy, xx, c])
    val = (p(ya, xa) * (1 - wx) + p(ya, xb) * wx) * (1 - wy) + (p(yb, xa) * (1 - wx) + p(yb, xb) * wx) * wy
    return val / 255.0
