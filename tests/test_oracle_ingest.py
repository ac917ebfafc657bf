"""Pins of the ingest oracle (letterbox + bilinear resize + /255) against
closed forms and a scalar evaluation."""

import numpy as np

from oracle.ingest import ingest, ingest_pixel, letterbox_geometry, resize_bilinear


def test_fullhd_letterbox_geometry():
    # 1920x1080 into 1088x608: r = 608/1080, the width rounds to 1081 and sits 3 px in
    assert letterbox_geometry(1080, 1920, 608, 1088) == (608, 1081, 0, 3)
    # same aspect: no border
    assert letterbox_geometry(1216, 2176, 608, 1088) == (608, 1088, 0, 0)
    # a 4:3 source is pillar-boxed
    nh, nw, top, left = letterbox_geometry(480, 640, 608, 1088)
    assert (nh, top) == (608, 0) and nw == round(640 * 608 / 480) and left == (1088 - nw) // 2


def test_identity_size_is_a_copy(rng):
    img = rng.integers(0, 256, (32, 48, 3))
    np.testing.assert_array_equal(resize_bilinear(img, 32, 48), img)


def test_halving_is_a_2x2_box_average(rng):
    img = rng.integers(0, 256, (16, 24, 3)).astype(np.float64)
    box = 0.25 * (img[0::2, 0::2] + img[1::2, 0::2] + img[0::2, 1::2] + img[1::2, 1::2])
    np.testing.assert_allclose(resize_bilinear(img, 8, 12), box, rtol=0, atol=1e-12)


def test_constant_and_linear_images():
    const = np.full((9, 13, 3), 77.0)
    np.testing.assert_allclose(resize_bilinear(const, 5, 7), 77.0, atol=1e-12)
    # a linear ramp in x is reproduced exactly where no clamping happens
    ramp = np.tile(np.arange(40.0)[None, :, None], (4, 1, 3))
    out = resize_bilinear(ramp, 4, 10)
    s = (np.arange(10) + 0.5) * 4.0 - 0.5
    np.testing.assert_allclose(out[0, :, 0], s, atol=1e-12)


def test_vectorised_equals_scalar_evaluation(rng):
    img = rng.integers(0, 256, (45, 80, 3)).astype(np.uint8)
    out = ingest(img, 64, 96)
    for _ in range(200):
        c, y, x = rng.integers(3), rng.integers(64), rng.integers(96)
        assert abs(out[c, y, x] - ingest_pixel(img, 64, 96, c, y, x)) <= 1e-12
    assert out.shape == (3, 64, 96) and out.min() >= 0.0 and out.max() <= 1.0
    nh, nw, top, left = letterbox_geometry(45, 80, 64, 96)
    assert np.all(out[:, :top] == 0.5) and np.all(out[:, top + nh:] == 0.5)
