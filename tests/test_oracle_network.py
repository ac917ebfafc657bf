"""Pins of the oracle's forward pass (CPU only).

Brute force on tiny tensors, closed-form special cases and structural
invariants; none of them re-types the oracle's own formula.
"""

import itertools

import numpy as np
import pytest

from jde_inputs import TINY, weight_specs, model_weights, tiny_frame, raw_weights, load_calib
from oracle import network as net


def brute_conv(x, w, b, stride):
    """Pure-Python loops over every output and every tap (zero padding k//2)."""
    n, h, wd, cin = x.shape
    cout, k, _, _ = w.shape
    p = k // 2
    ho = (h + 2 * p - k) // stride + 1
    wo = (wd + 2 * p - k) // stride + 1
    out = np.zeros((n, ho, wo, cout))
    for ni, y, xx, co in itertools.product(range(n), range(ho), range(wo), range(cout)):
        acc = float(b[co])
        for r, s, ci in itertools.product(range(k), range(k), range(cin)):
            iy, ix = y * stride + r - p, xx * stride + s - p
            if 0 <= iy < h and 0 <= ix < wd:
                acc += x[ni, iy, ix, ci] * w[co, r, s, ci]
        out[ni, y, xx, co] = acc
    return out


def im2col_conv(x, w, b, stride):
    """Independent formulation: gather patches into columns, one einsum."""
    n, h, wd, cin = x.shape
    cout, k, _, _ = w.shape
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    ho = (h + 2 * p - k) // stride + 1
    wo = (wd + 2 * p - k) // stride + 1
    cols = np.empty((n, ho, wo, k, k, cin))
    for y in range(ho):
        for xx in range(wo):
            cols[:, y, xx] = xp[:, y * stride:y * stride + k, xx * stride:xx * stride + k, :]
    return np.einsum("nyxrsc,orsc->nyxo", cols, w) + b


@pytest.mark.parametrize("k,stride,h,w,cin,cout", [
    (3, 1, 5, 7, 3, 4), (3, 2, 6, 8, 2, 3), (1, 1, 4, 5, 6, 2), (3, 2, 4, 4, 5, 5), (3, 1, 1, 1, 2, 3)])
def test_conv_matches_brute_force(rng, k, stride, h, w, cin, cout):
    x = rng.standard_normal((2, h, w, cin))
    wt = rng.standard_normal((cout, k, k, cin))
    b = rng.standard_normal(cout)
    ref = brute_conv(x, wt, b, stride)
    got = net.conv2d(x, wt, b, stride)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(im2col_conv(x, wt, b, stride), ref, rtol=1e-12, atol=1e-12)


def test_conv_1x1_is_matmul(rng):
    x = rng.standard_normal((2, 3, 4, 5))
    wt = rng.standard_normal((7, 1, 1, 5))
    got = net.conv2d(x, wt, None, 1)
    ref = np.einsum("nyxc,oc->nyxo", x, wt[:, 0, 0, :])
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_conv_delta_kernel_is_shift(rng):
    x = rng.standard_normal((1, 6, 7, 2))
    wt = np.zeros((2, 3, 3, 2))
    wt[0, 0, 2, 0] = 1.0     # out[y, x] = in[y - 1, x + 1]
    wt[1, 1, 1, 1] = 1.0     # identity on channel 1
    got = net.conv2d(x, wt, None, 1)
    shifted = np.zeros((6, 7))
    shifted[1:, :-1] = x[0, :-1, 1:, 0]
    np.testing.assert_array_equal(got[0, :, :, 0], shifted)
    np.testing.assert_array_equal(got[0, :, :, 1], x[0, :, :, 1])


def test_conv_stride2_is_subsampled_stride1(rng):
    x = rng.standard_normal((2, 8, 10, 3))
    wt = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    s1 = net.conv2d(x, wt, b, 1)
    s2 = net.conv2d(x, wt, b, 2)
    np.testing.assert_allclose(s2, s1[:, ::2, ::2, :], rtol=1e-12, atol=1e-12)


def test_elementwise_closed_forms():
    x = np.array([-2.0, -0.0, 0.0, 3.5])
    np.testing.assert_array_equal(net.leaky(x), [-0.2, 0.0, 0.0, 3.5])
    a = np.arange(2 * 2 * 3 * 1, dtype=float).reshape(2, 2, 3, 1)
    up = net.upsample2x(a)
    assert up.shape == (2, 4, 6, 1)
    for y in range(4):
        for xx in range(6):
            assert up[1, y, xx, 0] == a[1, y // 2, xx // 2, 0]
    c = net.concat(np.zeros((1, 1, 1, 2)), np.ones((1, 1, 1, 3)))
    np.testing.assert_array_equal(c[0, 0, 0], [0, 0, 1, 1, 1])


def _tiny_layers():
    return model_weights(TINY, 50)


def test_forward_layer_sequence_and_shapes():
    """Every conv runs once, in blob order, at the stride the topology gives it."""
    specs = weight_specs(TINY)
    seen = []
    frame = tiny_frame(TINY.seed, 0)[None]
    net.forward(frame, _tiny_layers(), TINY.blocks, pre_hook=lambda i, y: (seen.append((i, y.shape)), y)[1])
    assert [i for i, _ in seen] == list(range(len(specs)))
    stride = 1
    for (i, shape), (name, cout, k, cin, kind) in zip(seen, specs):
        if name.endswith(".down"):
            stride *= 2
        if name.startswith("p"):
            stride = int(name[1:name.index(".")])
        if name.startswith("lat"):
            stride = int(name[3:])
        assert shape == (1, 192 // stride, 320 // stride, cout), (name, shape)


def test_forward_concat_order_is_upsampled_then_skip():
    """Zero the skip-channel weights of p16.set0: its pre-activation must then be
    constant on 2x2 blocks (it sees only the upsampled lateral)."""
    specs = weight_specs(TINY)
    layers = [(w.copy(), b.copy()) for w, b in _tiny_layers()]
    i16 = [i for i, s in enumerate(specs) if s[0] == "p16.set0"][0]
    lat_c = specs[[i for i, s in enumerate(specs) if s[0] == "lat32"][0]][1]
    layers[i16][0][:, :, :, lat_c:] = 0.0
    got = {}
    net.forward(tiny_frame(TINY.seed, 0)[None], layers, TINY.blocks,
                pre_hook=lambda i, y: (got.__setitem__(i, y), y)[1])
    y = got[i16][0]
    assert np.abs(y).max() > 0.1
    np.testing.assert_array_equal(y[0::2, 0::2], y[1::2, 1::2])
    np.testing.assert_array_equal(y[0::2, 0::2], y[0::2, 1::2])


def test_forward_residual_after_activation_and_linear_outputs():
    """A block whose 3x3 conv outputs the constant -1 adds leaky(-1) = -0.1 to the
    stream; output convs with bias -1 and zero weights give exactly -1."""
    specs = weight_specs(TINY)
    layers = [(w.copy(), b.copy()) for w, b in _tiny_layers()]
    ic2 = [i for i, s in enumerate(specs) if s[0] == "s5.b0.c2"][0]
    layers[ic2][0][:] = 0.0
    layers[ic2][1][:] = -1.0
    for i, s in enumerate(specs):
        if s[4] in ("det", "emb"):
            layers[i][0][:] = 0.0
            layers[i][1][:] = -1.0
    got = {}
    out = net.forward(tiny_frame(TINY.seed, 0)[None], layers, TINY.blocks,
                      pre_hook=lambda i, y: (got.__setitem__(i, y), y)[1])
    down5 = got[[i for i, s in enumerate(specs) if s[0] == "s5.down"][0]]
    np.testing.assert_allclose(out["feat"][2], net.leaky(down5) - 0.1, rtol=0, atol=1e-15)
    for d in out["det"] + out["emb"]:
        assert np.all(d == -1.0)


def test_bn_fold_invariant():
    """On the calibration frame the folded conv's pre-activation has per-channel
    mean 0 and variance var / (var + eps)."""
    calib = load_calib(TINY)
    layers = model_weights(TINY, None, calib)
    kinds = [s[4] for s in weight_specs(TINY)]
    checked = []

    def hook(i, y):
        if kinds[i] == "bn":
            m = y.mean(axis=(0, 1, 2))
            v = y.var(axis=(0, 1, 2))
            ev = calib["var"][i] / (calib["var"][i] + 1e-5)
            assert np.abs(m).max() < 1e-4, (i, np.abs(m).max())
            np.testing.assert_allclose(v, ev, rtol=1e-4)
            checked.append(i)
        return y

    net.forward(tiny_frame(TINY.seed, 0)[None], layers, TINY.blocks, pre_hook=hook)
    assert len(checked) == kinds.count("bn")


def test_calibration_reproduces_stored_statistics():
    """The stored statistics are what calibrate_bn computes now (FP64, same seeds)."""
    calib = load_calib(TINY)
    kinds = [s[4] for s in weight_specs(TINY)]
    mu, var = net.calibrate_bn(tiny_frame(TINY.seed, 0)[None], raw_weights(TINY), TINY.blocks, kinds)
    for i in mu:
        np.testing.assert_allclose(mu[i], calib["mu"][i], rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(var[i], calib["var"][i], rtol=1e-9)


def test_rounding_models_match_library_casts_and_ties(rng):
    import torch
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-6, 6, 20000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    np.testing.assert_array_equal(net.round_bf16(x), ref)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert net.round_bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert net.round_bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6
    assert net.round_fp16(np.float32(1 + 2 ** -11)) == 1.0
    assert net.round_fp16(np.float32(1 + 3 * 2 ** -11)) == 1 + 2 ** -9
    assert np.isinf(net.round_bf16(np.float32(np.inf)))


def test_fp8_rounding_model_matches_library_cast_and_format(rng):
    """round_fp8 equals torch's float8_e4m3fn cast on every in-range value, and
    saturates at 448 where torch gives NaN; every e4m3 code point is a fixed point."""
    import torch
    x = (rng.standard_normal(50000) * 10.0 ** rng.uniform(-4, 2.6, 50000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float32).numpy().astype(np.float64)
    got = net.round_fp8(x)
    inr = np.abs(x) <= 448.0
    np.testing.assert_array_equal(got[inr], ref[inr])
    assert np.all(np.abs(got[~inr]) == 448.0)
    codes = torch.arange(0, 256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float32).numpy()
    codes = codes[np.isfinite(codes)].astype(np.float64)
    np.testing.assert_array_equal(net.round_fp8(codes), codes)
    assert len(np.unique(codes)) == 253          # 254 finite codes, +0 and -0 equal
    assert net.round_fp8(1.0625) == 1.0 and net.round_fp8(1.1875) == 1.25   # ties to even
    w = rng.standard_normal((5, 3, 3, 7))
    w[2] = 0.0
    wq, s = net.quantize_fp8_per_channel(w)
    assert s[2] == 1.0 and np.all(wq[2] == 0)
    np.testing.assert_allclose(np.abs(wq).reshape(5, -1).max(1)[[0, 1, 3, 4]],
                               np.abs(w).reshape(5, -1).max(1)[[0, 1, 3, 4]], rtol=1e-12)
    assert np.abs(wq - w).max() <= np.abs(w).max() / 16


def test_fp8_block_exponent_closed_forms():
    """The block exponent is the smallest s with max|x| / 2^s <= 448 (e4m3's
    largest value 1.75 * 2^8): hand-computed cases at and around the boundaries."""
    e = net.e8m0_exponent
    assert e(448.0) == 0 and e(np.nextafter(448.0, 0)) == 0
    assert e(np.nextafter(448.0, 1000)) == 1 and e(449.0) == 1 and e(896.0) == 1
    assert e(224.0) == -1 and e(224.5) == 0
    assert e(1.0) == -8          # 1 / 2^-8 = 256 <= 448, 1 / 2^-9 = 512 > 448
    assert e(1.75) == -8 and e(1.7500001) == -7
    assert e(0.0) == 0
    assert e(1e-300) == -127 and e(1e300) == 127        # the E8M0 range
    a = np.array([3.0, 0.0, 5e-5, 2.0 ** 20])
    want = [-7, 0, -23, 12]      # 3 / 2^-7 = 384; 5e-5 / 2^-23 = 419.4; 2^20 / 2^12 = 256
    np.testing.assert_array_equal(e(a), want)


def test_fp8_blocks_scale_each_block_on_its_own(rng):
    """quantize_fp8_blocks: every 32-value block along the last axis gets its own
    power of two (its largest magnitude lands in (224, 448] before rounding), a
    block's result does not depend on the other blocks, values 2^s * (e4m3 code)
    round-trip exactly, zero blocks stay zero, and the error of each value is at
    most half a unit of e4m3's top binade relative to its block's maximum."""
    x = rng.standard_normal((3, 5, 128)) * 10.0 ** rng.uniform(-6, 4, (3, 5, 1))
    x[1, 2, 32:64] = 0.0
    x[0, 0, 64:96] *= 1e-3                         # one block far below its neighbours
    q = net.quantize_fp8_blocks(x)
    xb, qb = x.reshape(3, 5, 4, 32), q.reshape(3, 5, 4, 32)
    amax = np.abs(xb).max(-1)
    s = net.e8m0_exponent(amax)
    nz = amax > 0
    top = np.ldexp(amax, -s)
    assert np.all((top[nz] > 224) & (top[nz] <= 448))
    assert np.all(qb[1, 2, 1] == 0)
    # a block's quantisation is the same alone as among others
    alone = net.quantize_fp8_blocks(x[0, 0, 64:96])
    np.testing.assert_array_equal(alone, q[0, 0, 64:96])
    # per-value error: <= 2^-4 of the block maximum (half a step of the top binade: 32 / 448 * 2^s ... bounded)
    err = np.abs(qb - xb).max(-1)
    assert np.all(err <= amax / 16 + 1e-300)
    # exact representables round-trip: 2^5 * e4m3 codes
    codes = np.array([448.0, -1.5, 0.0, 2.0 ** -9, 3.25, 288.0] + [1.0] * 26)
    np.testing.assert_array_equal(net.quantize_fp8_blocks(codes * 32.0), codes * 32.0)
    # the per-tensor e4m3 of the scaled-down block would flush it; the block scale keeps it
    assert np.abs(q[0, 0, 64:96] - x[0, 0, 64:96]).max() <= np.abs(x[0, 0, 64:96]).max() / 16


def test_fp8_weights_per_channel_and_block(rng):
    """quantize_fp8_per_channel_blocks: blocks run along the flattened (r, s, ci)
    order of each output channel, inside the channel scale max|w_c| / 448."""
    w = rng.standard_normal((4, 3, 3, 64))
    w[1] = 0.0
    w[2, 1, 1, :32] *= 1e-6                        # one 32-k block (tap (1, 1), ci 0..31) tiny
    wq, sc = net.quantize_fp8_per_channel_blocks(w)
    assert sc[1] == 1.0 and np.all(wq[1] == 0)
    np.testing.assert_allclose(sc[[0, 2, 3]], np.abs(w).reshape(4, -1).max(1)[[0, 2, 3]] / 448.0, rtol=1e-15)
    # the channel's largest weight is exact (it maps to 448)
    for c in (0, 2, 3):
        i = np.abs(w[c]).argmax()
        assert wq[c].flat[i] == w[c].flat[i]
    # the tiny block keeps its relative precision: error <= 1/16 of its own maximum
    blk = w[2, 1, 1, :32]
    assert np.abs(wq[2, 1, 1, :32] - blk).max() <= np.abs(blk).max() / 16
    # with one scale per channel only, the same block would lose almost everything
    wq1, _ = net.quantize_fp8_per_channel(w)
    assert np.abs(wq1[2, 1, 1, :32] - blk).max() > 10 * np.abs(wq[2, 1, 1, :32] - blk).max()


def _codes(e_bits, m_bits, bias):
    """Every non-negative value of a sign / e_bits / m_bits minifloat with no inf or
    NaN codes, from its definition: exponent field E = 0 is subnormal
    (m / 2^M * 2^(1 - bias)), else (1 + m / 2^M) * 2^(E - bias); with the
    mantissa's lowest bit (the tie-break parity)."""
    out = []
    for E in range(2 ** e_bits):
        for m in range(2 ** m_bits):
            v = (m / 2 ** m_bits) * 2.0 ** (1 - bias) if E == 0 else (1 + m / 2 ** m_bits) * 2.0 ** (E - bias)
            out.append((v, m & 1))
    return sorted(out)


@pytest.mark.parametrize("fmt,e_bits,m_bits,bias", [("fp4", 2, 1, 1), ("fp6", 2, 3, 1)])
def test_fp4_fp6_rounding_is_nearest_code_ties_to_even(rng, fmt, e_bits, m_bits, bias):
    """round_minifloat against brute force over the format's codes: the nearest
    representable value, ties to the code whose mantissa is even, saturating at the
    largest code; exact at every code and at hand-picked ties."""
    codes = _codes(e_bits, m_bits, bias)
    vals = np.array([v for v, _ in codes])
    assert vals.max() == net.MINIFLOATS[fmt][2]
    x = np.concatenate([rng.uniform(-9, 9, 4000), vals, -vals, (vals[1:] + vals[:-1]) / 2])
    want = []
    for xi in x:
        a = min(abs(xi), vals.max())
        d = np.abs(vals - a)
        best = np.flatnonzero(d == d.min())
        if len(best) > 1:                      # a tie: the even-mantissa code
            best = [b for b in best if codes[b][1] == 0]
        want.append(np.sign(xi) * vals[best[0]])
    np.testing.assert_array_equal(net.round_minifloat(x, fmt), np.array(want))
    if fmt == "fp4":
        got = net.round_minifloat(np.array([0.25, 0.75, 1.25, 1.75, 2.5, 3.5, 5.0, 7.0]), "fp4")
        np.testing.assert_array_equal(got, [0.0, 1.0, 1.0, 2.0, 2.0, 4.0, 4.0, 6.0])


def test_fp4_fp6_block_exponents_and_blocks(rng):
    """Block exponents against each format's largest value (6 for FP4, 7.5 for FP6
    E2M3), and block quantisation that scales each 32-value block on its own."""
    e = net.e8m0_exponent
    assert e(6.0, 6.0) == 0 and e(6.0001, 6.0) == 1 and e(3.0, 6.0) == -1 and e(3.1, 6.0) == 0
    assert e(7.5, 7.5) == 0 and e(1.0, 7.5) == -2      # 1 / 2^-2 = 4 <= 7.5 < 8 = 1 / 2^-3
    for fmt in ("fp4", "fp6"):
        top = net.MINIFLOATS[fmt][2]
        x = rng.standard_normal((4, 64)) * 10.0 ** rng.uniform(-3, 3, (4, 1))
        q = net.quantize_blocks(x, fmt)
        xb, qb = x.reshape(4, 2, 32), q.reshape(4, 2, 32)
        s = net.e8m0_exponent(np.abs(xb).max(-1), top)
        t = np.ldexp(np.abs(xb).max(-1), -s)
        assert np.all((t > top / 2) & (t <= top))
        np.testing.assert_array_equal(net.quantize_blocks(x[1, 32:], fmt), q[1, 32:])
        # every quantised value is 2^s times a code of the format
        np.testing.assert_array_equal(net.round_minifloat(np.ldexp(qb, -s[..., None]), fmt), np.ldexp(qb, -s[..., None]))
