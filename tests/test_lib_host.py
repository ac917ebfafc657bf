"""CPU tests of libjde: exported symbols, layer plan, argument checks, and the
host FP64 association code (Kalman filter, assignment) against the oracle.

No device work is enqueued here: every call either is host code or fails its
argument checks before touching the GPU.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from jde_inputs import TINY, FULL, weight_specs, anchors_px
from oracle import track as otrack

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2011_03910_amd import _lib
    return _lib.load()


def header_functions():
    src = open(os.path.join(ROOT, "include", "jde.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(jde_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(lib):
    from paper_2011_03910_amd import _lib
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, n
    nm = os.popen(f"nm -D --defined-only {_lib.LIB_PATH}").read()
    for n in names:
        assert re.search(rf"\bT {n}\b", nm), n


@pytest.mark.parametrize("cfg", [TINY, FULL])
def test_layer_plan_matches_weight_blob_order(cfg):
    import paper_2011_03910_amd as P
    ctx = P.jde_create(cfg.c0, cfg.blocks, cfg.emb_dim, anchors_px(cfg), "bf16", 2, cfg.height, cfg.width, 512)
    try:
        from paper_2011_03910_amd import _lib
        L = _lib.load()
        shapes = [P.jde_layer_info(ctx, i) for i in range(L.jde_num_layers(ctx))]
        specs = weight_specs(cfg)
        assert [(s[1], s[2], s[3]) for s in specs] == [(a, b, c) for a, b, c, _ in shapes]
        assert L.jde_blob_floats(ctx) == sum(co * k * k * ci + co for _, co, k, ci, _ in specs)
        strides = [st for *_, st in shapes]
        assert strides.count(2) == 5
    finally:
        P.jde_destroy(ctx)


def _cfg(**kw):
    from paper_2011_03910_amd import _lib
    c = _lib.JdeConfig()
    c.base_ch, c.emb_dim, c.num_anchors, c.precision = 16, 64, 4, 0
    for i, b in enumerate(TINY.blocks):
        c.blocks[i] = b
    c.max_frames, c.max_h, c.max_w, c.max_candidates = 2, 192, 320, 256
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("kw,status", [
    (dict(num_anchors=3), -5), (dict(precision=7), -5), (dict(max_h=100), -1), (dict(max_frames=0), -1),
    (dict(max_frames=65), -1), (dict(max_candidates=100), -1), (dict(max_candidates=16384), -1),
    (dict(emb_dim=60), -1), (dict(base_ch=24), -5)])
def test_create_rejects_bad_configs(lib, kw, status):
    h = ctypes.c_void_p()
    assert lib.jde_create(ctypes.byref(_cfg(**kw)), ctypes.byref(h)) == status
    assert lib.jde_last_error()


def test_calls_fail_before_device_work(lib):
    from paper_2011_03910_amd import _lib
    h = ctypes.c_void_p()
    assert lib.jde_create(ctypes.byref(_cfg()), ctypes.byref(h)) == 0
    try:
        d = (_lib.JdeFrameDesc * 3)()
        for i in range(3):
            d[i].h, d[i].w = 192, 320
        heads = _lib.JdeHeadOut()
        ws = lib.jde_workspace_bytes(h)
        fake = ctypes.c_void_p(0x1000)
        # forward before weights are loaded
        assert lib.jde_forward(h, fake, d, 1, fake, ws, ctypes.byref(heads), None) == _lib.JDE_ESTATE
        # wrong blob size
        assert lib.jde_load_weights(h, None, 5, fake, 10, None) == _lib.JDE_EINVAL
        blob = np.zeros(lib.jde_blob_floats(h), dtype=np.float32)
        assert lib.jde_load_weights(h, blob.ctypes.data_as(_lib.c_float_p), blob.size, fake, 10,
                                    None) == _lib.JDE_ENOMEM
        # too many frames / bad frame size / small workspace / cap mismatch
        dets = _lib.JdeDets()
        assert lib.jde_decode(h, ctypes.byref(heads), d, 3, 0.5, 0.4, None, fake, ws, ctypes.byref(dets),
                              None) == _lib.JDE_EINVAL
        dets.cap = 256
        for k in ("boxes", "scores", "margins", "emb", "anchor_idx", "count", "n_cand", "overflow"):
            setattr(dets, k, 0x1000)
        assert lib.jde_decode(h, ctypes.byref(heads), d, 3, 0.5, 0.4, None, fake, ws, ctypes.byref(dets),
                              None) == _lib.JDE_ECAPACITY
        d[0].h = 100
        assert lib.jde_decode(h, ctypes.byref(heads), d, 1, 0.5, 0.4, None, fake, ws, ctypes.byref(dets),
                              None) == _lib.JDE_EINVAL
        d[0].h = 192
        assert lib.jde_decode(h, ctypes.byref(heads), d, 1, 0.5, 0.4, None, fake, ws - 1, ctypes.byref(dets),
                              None) == _lib.JDE_ENOMEM
        assert lib.jde_decode(h, ctypes.byref(heads), d, 1, 1.5, 0.4, None, fake, ws, ctypes.byref(dets),
                              None) == _lib.JDE_EINVAL
        assert lib.jde_nms(h, fake, fake, fake, 257, 0.4, fake, ws, fake, fake, None) == _lib.JDE_ECAPACITY
        assert lib.jde_cost_matrix(None, None, None, 3, None, None, 4, 64, 9.4877, None, None) == _lib.JDE_EINVAL
        assert lib.jde_cost_matrix(None, None, None, 3, None, None, 4, 62, 9.4877, None, None) == _lib.JDE_EINVAL
        sizes = (ctypes.c_size_t * 3)(), (ctypes.c_size_t * 3)()
        assert lib.jde_head_sizes(h, d, 2, *sizes) == 0
        assert sizes[0][0] == 2 * 24 * 40 * 24 and sizes[1][2] == 2 * 6 * 10 * 64
    finally:
        lib.jde_destroy(h)


def test_kalman_matches_oracle(rng):
    import paper_2011_03910_amd as P
    z = np.array([300.0, 200.0, 0.45, 120.0])
    m, c = P.jde_kf_initiate(z)
    mo, co = otrack.kf_initiate(z)
    np.testing.assert_array_equal(m, mo)
    np.testing.assert_array_equal(c, co)
    for step in range(50):
        mm = m[None].copy()
        cc = c[None].copy()
        P.jde_kf_predict(mm, cc)
        mo, co = otrack.kf_predict(mo, co)
        np.testing.assert_allclose(mm[0], mo, rtol=1e-14, atol=1e-12)
        np.testing.assert_allclose(cc[0], co, rtol=1e-12, atol=1e-12)
        zz = mo[:4] + rng.normal(0, 1, 4) * [3, 3, 0.01, 2]
        m, c = P.jde_kf_update(mm[0], cc[0], zz)
        mo, co = otrack.kf_update(mo, co, zz)
        np.testing.assert_allclose(m, mo, rtol=1e-10, atol=1e-9)
        np.testing.assert_allclose(c, co, rtol=1e-8, atol=1e-9)
        assert np.array_equal(c, c.T)
        m, c = mo.copy(), co.copy()


def test_batched_kalman_update_matches_oracle(rng):
    """jde_kf_update_n applies the oracle's update to exactly the listed tracks."""
    import paper_2011_03910_amd as P
    T = 7
    zs0 = np.column_stack([rng.uniform(100, 900, T), rng.uniform(100, 500, T), rng.uniform(0.3, 0.6, T),
                           rng.uniform(40, 200, T)])
    mean, cov = P.jde_kf_initiate_n(zs0)
    P.jde_kf_predict(mean, cov)
    z = zs0[[3, 1, 0]] + rng.normal(0, 1, (3, 4)) * [3, 3, 0.01, 2]
    ti, di = np.array([4, 0, 6]), np.array([0, 2, 1])
    m1, c1 = mean.copy(), cov.copy()
    P.jde_kf_update_n(ti, di, m1, c1, z)
    for t in range(T):
        if t in ti:
            d = di[list(ti).index(t)]
            mo, co = otrack.kf_update(mean[t], cov[t], z[d])
            np.testing.assert_allclose(m1[t], mo, rtol=1e-10, atol=1e-9)
            np.testing.assert_allclose(c1[t], co, rtol=1e-8, atol=1e-9)
        else:
            np.testing.assert_array_equal(m1[t], mean[t])
            np.testing.assert_array_equal(c1[t], cov[t])
    P.jde_kf_update_n(np.zeros(0, int), np.zeros(0, int), m1, c1, z)


@pytest.mark.parametrize("t_n,d_n", [(5, 5), (8, 13), (13, 8), (1, 1), (0, 4), (60, 45), (200, 200)])
def test_assign_matches_oracle(rng, t_n, d_n):
    import paper_2011_03910_amd as P
    for _ in range(3):
        c = rng.uniform(0, 1.3, (t_n, d_n)).astype(np.float32)
        if c.size:
            c[rng.random(c.shape) < 0.4] = np.inf
        pairs, total = P.jde_assign(c, 0.7)
        rp, rt = otrack.assign(c.astype(np.float64), 0.7)
        assert len(pairs) == len(rp)
        assert total == pytest.approx(rt, abs=1e-9)
        if len(pairs):
            assert np.all(c[pairs[:, 0], pairs[:, 1]] <= 0.7)
            assert len(set(pairs[:, 1])) == len(pairs)


def test_assign_with_forbidden_rows_and_columns_matches_oracle(rng):
    """Tracks or detections with no allowed entry can never be matched; the
    assignment (which drops them before its search) still equals the oracle's."""
    import paper_2011_03910_amd as P
    for T, D in ((30, 12), (12, 30), (25, 25)):
        for trial in range(4):
            c = rng.uniform(0, 1.3, (T, D)).astype(np.float32)
            c[rng.random(T) < 0.5, :] = np.inf          # whole tracks forbidden
            c[:, rng.random(D) < 0.3] = np.inf          # whole detections forbidden
            c[rng.random(c.shape) < 0.3] = np.inf
            pairs, total = P.jde_assign(c, 0.7)
            rp, rt = otrack.assign(c.astype(np.float64), 0.7)
            assert len(pairs) == len(rp) and total == pytest.approx(rt, abs=1e-9)
    assert len(P.jde_assign(np.full((40, 9), np.inf, np.float32), 0.7)[0]) == 0
    one = np.full((50, 20), np.inf, np.float32)
    one[17, 3] = 0.25
    pairs, total = P.jde_assign(one, 0.7)
    assert pairs.tolist() == [[17, 3]] and total == pytest.approx(0.25)


def test_fp8_encoder_matches_library_cast():
    """The weight encoder (host, product) equals torch's float8_e4m3fn cast on
    in-range values, saturates to 448 and maps NaN to 0x7f."""
    import torch
    import paper_2011_03910_amd as P
    from paper_2011_03910_amd.jde import jde_fp8_encode
    r = np.random.Generator(np.random.PCG64(88))
    x = (r.standard_normal(40000) * 10.0 ** r.uniform(-5, 2.6, 40000)).astype(np.float32)
    x[:6] = [0.0, -0.0, 448.0, -448.0, 2 ** -9, 1.0625]
    got = jde_fp8_encode(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    inr = np.abs(x) <= 448.0
    np.testing.assert_array_equal(got[inr], ref[inr])
    big = np.array([449.0, 1e9, -600.0, np.nan], dtype=np.float32)
    np.testing.assert_array_equal(jde_fp8_encode(big), [0x7E, 0x7E, 0xFE, 0x7F])


@pytest.mark.parametrize("fmt,e_bits,m_bits", [("fp6", 2, 3), ("fp4", 2, 1)])
def test_fp6_fp4_encoder_matches_the_oracle_rounding(fmt, e_bits, m_bits):
    """The FP6 E2M3 / FP4 E2M1 weight encoder (host, product): its codes, decoded
    by the format's definition (bias 1: E = 0 is m / 2^M, else (1 + m / 2^M)
    2^(E - 1)), equal the oracle's nearest-even rounding with saturation, on random
    values, every tie point between neighbouring codes and out-of-range values."""
    from oracle.network import round_minifloat
    from paper_2011_03910_amd.jde import jde_mx_encode
    r = np.random.Generator(np.random.PCG64(89))
    x = (r.standard_normal(20000) * 10.0 ** r.uniform(-3, 1.2, 20000)).astype(np.float32)
    grid = np.unique(np.abs(round_minifloat(np.linspace(0, 8, 4001), fmt)))
    x = np.concatenate([x, grid, -grid, (grid[1:] + grid[:-1]) / 2, [9.0, -1e6, 0.0, -0.0]]).astype(np.float32)
    codes = jde_mx_encode(fmt, x).astype(np.int64)
    bits = 1 + e_bits + m_bits
    sign = np.where((codes >> (bits - 1)) & 1, -1.0, 1.0)
    E = (codes >> m_bits) & ((1 << e_bits) - 1)
    m = codes & ((1 << m_bits) - 1)
    val = np.where(E == 0, m / 2.0 ** m_bits, (1 + m / 2.0 ** m_bits) * 2.0 ** (E - 1.0)) * sign
    assert codes.max() < (1 << bits)
    np.testing.assert_array_equal(val, round_minifloat(x.astype(np.float64), fmt))


def test_nms_noalloc_rejects_lists_beyond_its_scratch(lib):
    """The static-scratch NMS refuses K > 8192 before any device work."""
    from paper_2011_03910_amd import _lib
    st = lib.jde_nms_noalloc(None, None, None, 8193, ctypes.c_float(0.4), ctypes.c_void_p(16),
                             ctypes.c_void_p(16), None)
    assert st == _lib.JDE_ECAPACITY
    assert "8192" in lib.jde_last_error().decode()
    assert lib.jde_nms_noalloc(None, None, None, -1, ctypes.c_float(0.4), ctypes.c_void_p(16),
                               ctypes.c_void_p(16), None) == _lib.JDE_EINVAL


def test_box_to_z_matches_oracle(rng):
    from paper_2011_03910_amd import jde_box_to_z
    xy = rng.uniform(0, 1000, (50, 2))
    wh = rng.uniform(5, 300, (50, 2))
    boxes = np.concatenate([xy, xy + wh], 1).astype(np.float32)
    got = jde_box_to_z(boxes)
    want = np.stack([otrack.box_to_z(b) for b in boxes.astype(np.float64)])
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=0)


def test_frame_bytes_and_budget_admission():
    """jde_frame_bytes adds up a frame's pixels, heads, detection rows and its
    pixel share of the workspace; jde_admit admits the longest prefix within the
    budget and refuses with JDE_EBUDGET when even the first frame does not fit."""
    import paper_2011_03910_amd as P
    from paper_2011_03910_amd import _lib
    L = _lib.load()
    ctx = P.jde_create(FULL.c0, FULL.blocks, FULL.emb_dim, anchors_px(FULL), "bf16", 8, 608, 1088, 512)
    try:
        fb = lambda h, w: L.jde_frame_bytes(ctx, h, w)
        big, mid, small = fb(608, 1088), fb(480, 864), fb(320, 576)
        heads = sum((608 >> (3 + s)) * (1088 >> (3 + s)) * (24 + 512) * 4 for s in range(3))
        share = L.jde_workspace_bytes(ctx) / 8
        assert big >= 3 * 608 * 1088 * 4 + heads + share
        assert big > mid > small > 0
        assert fb(600, 1088) == 0 and fb(640, 1088) == 0
        descs = (_lib.JdeFrameDesc * 4)()
        for i, (h, w) in enumerate(((608, 1088), (320, 576), (480, 864), (608, 1088))):
            descs[i].h, descs[i].w = h, w
        n = ctypes.c_int(-1)
        assert L.jde_admit(ctx, descs, 4, 0, big + small + mid, ctypes.byref(n)) == 0 and n.value == 3
        assert L.jde_admit(ctx, descs, 4, 0, big + small + mid - 1, ctypes.byref(n)) == 0 and n.value == 2
        assert L.jde_admit(ctx, descs, 4, 10 ** 12, 2 * 10 ** 12, ctypes.byref(n)) == 0 and n.value == 4
        assert L.jde_admit(ctx, descs, 4, 5, big + 4, ctypes.byref(n)) == _lib.JDE_EBUDGET and n.value == 0
        assert "budget" in L.jde_last_error().decode()
        descs[1].h = 100
        assert L.jde_admit(ctx, descs, 4, 0, 10 ** 12, ctypes.byref(n)) == _lib.JDE_EINVAL
    finally:
        P.jde_destroy(ctx)
