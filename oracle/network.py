"""FP64 oracle of the JDE forward pass (test infrastructure only).

The paper describes the model as a Darknet-53 backbone with detection done the
YOLOv3 way, an FPN in which higher-level features are upsampled and fused with
lower-level ones, and prediction heads on three layers (Sec. 3.1).  The exact
head layout is not given; the reading used here (and by the product) is:

* backbone: stem 3x3 conv, then five stages of [3x3 stride-2 conv, residual
  blocks x + leaky(conv3x3(leaky(conv1x1(x))))]; C3/C4/C5 are the stage 3/4/5
  outputs (strides 8/16/32);
* each head: five convs (1x1, 3x3, 1x1, 3x3, 1x1) to a feature F, a det branch
  (3x3 then a linear 1x1 to 6 outputs per anchor) and a linear 3x3 emb branch;
* a lateral 1x1 from F, nearest x2 upsample, concat [upsampled, skip] feeds the
  next finer head.

Every non-output conv is conv + folded batch-norm bias, then leaky ReLU 0.1;
the residual add comes after the activation.  Output convs are linear + bias.
"""

import numpy as np

LEAKY_SLOPE = 0.1
BN_EPS = 1e-5


def conv2d(x, w, b, stride):
    """Direct convolution, zero padding k//2.

    out[n, y, x, co] = b[co] + sum_{r, s, ci} in[n, y*st + r - p, x*st + s - p, ci] * w[co, r, s, ci]

    x: [N, H, W, Cin] FP64 NHWC.  w: [Cout, k, k, Cin].  b: [Cout] or None.
    The sum over ci of each tap is one matmul; taps are added in (r, s) order.
    """
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, h, wd, cin = x.shape
    cout, k, k2, cin_w = w.shape
    assert k == k2 and cin == cin_w, (x.shape, w.shape)
    p = k // 2
    ho = (h + 2 * p - k) // stride + 1
    wo = (wd + 2 * p - k) // stride + 1
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    out = np.zeros((n * ho * wo, cout))
    for r in range(k):
        for s in range(k):
            tap = xp[:, r:r + stride * (ho - 1) + 1:stride, s:s + stride * (wo - 1) + 1:stride, :]
            out += tap.reshape(-1, cin) @ w[:, r, s, :].T
    out = out.reshape(n, ho, wo, cout)
    if b is not None:
        out = out + np.asarray(b, dtype=np.float64)
    return out


def leaky(x):
    """Leaky ReLU with slope 0.1 (x > 0 ? x : 0.1 x)."""
    return np.where(x > 0, x, LEAKY_SLOPE * x)


def upsample2x(x):
    """Nearest x2: up[n, y, x, c] = in[n, y // 2, x // 2, c]."""
    return x.repeat(2, axis=1).repeat(2, axis=2)


def concat(a, b):
    """Channel concat in the order [a, b]."""
    return np.concatenate([a, b], axis=3)


def ingest(frames):
    """[N, 3, H, W] pixels -> [N, H, W, 3] FP64 (layout change only)."""
    return np.ascontiguousarray(np.asarray(frames, dtype=np.float64).transpose(0, 2, 3, 1))


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def round_fp16(x):
    """Round to the nearest IEEE half (ties to even), returned as FP64."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


FP8_MAX = 448.0


def round_fp8(x):
    """Round to the nearest OCP FP8 e4m3 value (ties to even), saturating at +-448.

    e4m3: 3 mantissa bits; normal binades 2^-6 .. 2^8 have spacing 2^(e-3);
    below 2^-6 the subnormal spacing is 2^-9.  Returned as FP64.
    """
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), FP8_MAX)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)
    q = np.exp2(e - 3.0)
    r = np.round(a / q) * q            # numpy rounds halves to even
    r = np.minimum(r, FP8_MAX)
    return np.where(np.isnan(x), np.nan, np.sign(x) * r)


def quantize_fp8_per_channel(w):
    """Per-output-channel symmetric FP8 quantisation of w [Cout, ...]:
    s_c = max|w_c| / 448 (1 for an all-zero channel), w ~= s_c * round_fp8(w / s_c).
    Returns (dequantised weights, scales)."""
    w = np.asarray(w, dtype=np.float64)
    amax = np.abs(w.reshape(w.shape[0], -1)).max(axis=1)
    s = np.where(amax > 0, amax / FP8_MAX, 1.0)
    sb = s.reshape((-1,) + (1,) * (w.ndim - 1))
    return round_fp8(w / sb) * sb, s


# The element formats of the block-scaled matrix-core operands (OCP microscaling):
# mantissa bits M, smallest normal exponent emin (bias 1 - emin), largest value.
# e4m3: 3 mantissa bits, exponent bias 7, max 1.75 * 2^8; FP6 E2M3: 3 mantissa bits,
# bias 1, max 1.875 * 2^2; FP4 E2M1: 1 mantissa bit, bias 1, max 1.5 * 2^2.
MINIFLOATS = {"fp8": (3, -6, 448.0), "fp6": (3, 0, 7.5), "fp4": (1, 0, 6.0)}


def round_minifloat(x, fmt):
    """Round to the nearest value of the element format ``fmt`` (ties to even),
    saturating at its largest value; the spacing in binade e >= emin is 2^(e - M),
    below 2^emin it stays 2^(emin - M) (subnormals).  Returned as FP64."""
    mant, emin, top = MINIFLOATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), top)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, float(emin))
    q = np.exp2(e - mant)
    r = np.minimum(np.round(a / q) * q, top)     # numpy rounds halves to even
    return np.where(np.isnan(x), np.nan, np.sign(x) * r)


def e8m0_exponent(amax, top=FP8_MAX):
    """Power-of-two block scale with 32-value blocks (the E8M0 scale the matrix
    cores apply): the smallest integer s with amax / 2^s <= top (the element
    format's largest value, 448 for e4m3), so that the block's largest magnitude
    lands in the format's top binade without saturating; s = 0 for an all-zero
    block; s is kept within the E8M0 range [-127, 127]."""
    a = np.asarray(amax, dtype=np.float64)
    pos = a > 0
    s = np.ceil(np.log2(np.where(pos, a, top) / top))
    # log2 is inexact near powers of two: settle s with exact power-of-two scalings
    s = np.where(np.ldexp(np.where(pos, a, 0.0), -s.astype(np.int64)) > top, s + 1, s)
    s = np.where(np.ldexp(np.where(pos, a, 0.0), -(s - 1).astype(np.int64)) <= top, s - 1, s)
    s = np.where(pos, s, 0.0)
    return np.clip(s, -127, 127).astype(np.int64)


def quantize_blocks(x, fmt="fp8", block=32):
    """Element format ``fmt`` with a power-of-two scale per block of ``block``
    consecutive values along the last axis: each block b becomes
    2^s_b round(x / 2^s_b) with s_b = e8m0_exponent(max |x_b|, top of fmt).  The
    last axis must be a multiple of block.  Returns the dequantised values (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    assert x.shape[-1] % block == 0, x.shape
    xb = x.reshape(x.shape[:-1] + (x.shape[-1] // block, block))
    s = e8m0_exponent(np.abs(xb).max(axis=-1), MINIFLOATS[fmt][2])[..., None]
    return (np.ldexp(round_minifloat(np.ldexp(xb, -s), fmt), s)).reshape(x.shape)


def quantize_fp8_blocks(x, block=32):
    """e4m3 with a power-of-two scale per block (quantize_blocks with 'fp8')."""
    return quantize_blocks(x, "fp8", block)


def quantize_per_channel_blocks(w, fmt="fp8", block=32):
    """Block-scaled weights with a per-output-channel scale and, inside it, a
    power-of-two scale per block of 32 along the flattened (r, s, ci) axis of
    w [Cout, k, k, Cin]: w ~= s_c * 2^s_cb * round(w / s_c / 2^s_cb),
    s_c = max|w_c| / top of fmt.  Returns (dequantised weights, per-channel scales)."""
    top = MINIFLOATS[fmt][2]
    w = np.asarray(w, dtype=np.float64)
    amax = np.abs(w.reshape(w.shape[0], -1)).max(axis=1)
    s = np.where(amax > 0, amax / top, 1.0)
    flat = w.reshape(w.shape[0], -1) / s[:, None]
    return (quantize_blocks(flat, fmt, block) * s[:, None]).reshape(w.shape), s


def quantize_fp8_per_channel_blocks(w, block=32):
    """quantize_per_channel_blocks with e4m3 elements."""
    return quantize_per_channel_blocks(w, "fp8", block)


class _Walker:
    """Consumes the weight list in blob order (see jde_inputs.weights)."""

    def __init__(self, layers, pre_hook, store, in_hook):
        self.layers = layers
        self.i = 0
        self.pre_hook = pre_hook
        self.store = store
        self.in_hook = in_hook

    def conv(self, x, stride=1, act=True, res=None):
        w, b = self.layers[self.i]
        xin = x if self.in_hook is None else self.in_hook(self.i, x)
        y = conv2d(xin, w, b, stride)
        if self.pre_hook is not None:
            y = self.pre_hook(self.i, y)
        self.i += 1
        if act:
            y = leaky(y)
        if res is not None:
            y = y + res
        if act and self.store is not None:
            y = self.store(y)
        return y


def forward(frames, layers, blocks, pre_hook=None, store=None, in_hook=None):
    """JDE forward (Sec. 3.1).

    frames: [N, 3, H, W] (H, W divisible by 32).  layers: list of (w, b) in blob
    order.  blocks: residual blocks per stage.  pre_hook(i, pre) may rewrite the
    pre-activation of conv i (used by the batch-norm calibration).  store(y), if
    given, is applied to every activation a non-output conv stores (after its
    activation and residual add): round_bf16 / round_fp16 model a network whose
    activations are kept in that format (the exact arithmetic stays FP64).
    in_hook(i, x), if given, replaces the input conv i reads (the residual and
    the stored tensor are unchanged): it models an input quantised for conv i.

    Returns dict with 'det' = [d8, d16, d32] ([N, H/s, W/s, 6A]) and
    'emb' = [e8, e16, e32] ([N, H/s, W/s, E]), all FP64, plus 'feat' = C3, C4, C5.
    """
    nb = _Walker(layers, pre_hook, store, in_hook)
    x = ingest(frames)
    x = nb.conv(x)                                   # stem
    feats = {}
    for s, nblk in enumerate(blocks, 1):
        x = nb.conv(x, stride=2)                     # downsample
        for _ in range(nblk):
            y = nb.conv(x)                           # 1x1 C -> C/2
            x = nb.conv(y, res=x)                    # 3x3 C/2 -> C, + x after leaky
        feats[s] = x
    det, emb = {}, {}
    lat = None
    for lvl, stage in ((32, 5), (16, 4), (8, 3)):
        x = feats[stage] if lat is None else concat(upsample2x(lat), feats[stage])
        for _ in range(5):
            x = nb.conv(x)                           # 1x1, 3x3, 1x1, 3x3, 1x1
        d = nb.conv(x)                               # det 3x3
        det[lvl] = nb.conv(d, act=False)             # det 1x1 (linear)
        emb[lvl] = nb.conv(x, act=False)             # emb 3x3 (linear)
        if lvl != 8:
            lat = nb.conv(x)                         # lateral 1x1
    assert nb.i == len(layers), (nb.i, len(layers))
    return {"det": [det[8], det[16], det[32]], "emb": [emb[8], emb[16], emb[32]],
            "feat": [feats[3], feats[4], feats[5]]}


def calibrate_bn(frames, raw_layers, blocks, kinds):
    """Batch-norm statistics of the synthetic network (stand-in for training).

    Runs the forward with the raw weights (zero bias).  For every conv whose kind
    is 'bn', in forward order, the per-channel mean and (population) variance of
    its pre-activation over (n, y, x) are recorded, and the pre-activation is
    replaced by (pre - mean) / sqrt(var + eps) before the activation, which is
    exactly the folded conv w / sqrt(var + eps), bias -mean / sqrt(var + eps).
    Returns (mu, var) dicts keyed by conv index.
    """
    mu, var = {}, {}

    def hook(i, pre):
        if kinds[i] != "bn":
            return pre
        m = pre.mean(axis=(0, 1, 2))
        v = ((pre - m) ** 2).mean(axis=(0, 1, 2))
        mu[i], var[i] = m, v
        return (pre - m) / np.sqrt(v + BN_EPS)

    layers = [(w, np.zeros(w.shape[0])) for w in raw_layers]
    forward(frames, layers, blocks, pre_hook=hook)
    return mu, var
