"""Pins of the oracle's cost matrix, gate, Kalman filter and assignment (CPU only)."""

import itertools
import json
import math
import os

import numpy as np
import pytest

from jde_inputs import synthetic_dets_tracks
from oracle import track as tk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_cosine_closed_forms():
    f = np.eye(4)[:3]
    e = np.stack([np.eye(4)[0], np.eye(4)[1], -np.eye(4)[2], np.eye(4)[3]])
    mean = np.tile([[50.0, 50.0, 0.5, 100.0, 0, 0, 0, 0]], (3, 1))
    cov = np.tile(np.eye(8) * 1e6, (3, 1, 1))                    # gate never fires
    boxes = np.tile([[25.0, 0.0, 75.0, 100.0]], (4, 1))
    c = tk.cost_matrix(f, mean, cov, boxes, e)
    np.testing.assert_array_equal(c, [[0, 1, 1, 1], [1, 0, 1, 1], [1, 1, 2, 1]])


def test_chi2_gate_constant_closed_form():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["chi2_4dof_95"]
    x = tk.CHI2_4_95
    assert x == g["value"]
    cdf = 1.0 - math.exp(-x / 2.0) * (1.0 + x / 2.0)            # chi-square CDF, 4 dof
    assert abs(cdf - g["cdf_at_value"]) < 2e-5


def test_gate_passes_95_percent_of_own_distribution(rng):
    mean = np.array([300.0, 200.0, 0.4, 150.0, 1, 1, 0, 0])
    a = rng.standard_normal((8, 8))
    cov = a @ a.T + np.eye(8)
    hx, s = tk.kf_project(mean, cov)
    z = rng.multivariate_normal(hx, s, 40000)
    d2 = tk.mahalanobis_sq(mean, cov, z)
    assert abs((d2 <= tk.CHI2_4_95).mean() - 0.95) < 0.005


def test_mahalanobis_reduces_to_euclidean_and_matches_inverse(rng):
    mean = np.array([10.0, 20.0, 0.5, 40.0, 0, 0, 0, 0])
    r = tk.measurement_noise(mean)
    cov = np.eye(8)
    cov[:4, :4] = np.eye(4) - r                                   # S = H P H^T + R = I
    z = rng.standard_normal((30, 4)) + mean[:4]
    np.testing.assert_allclose(tk.mahalanobis_sq(mean, cov, z), ((z - mean[:4]) ** 2).sum(1), rtol=1e-12)
    a = rng.standard_normal((8, 8))
    cov = a @ a.T + 0.1 * np.eye(8)
    _, s = tk.kf_project(mean, cov)
    y = z - mean[:4]
    ref = np.einsum("di,ij,dj->d", y, np.linalg.inv(s), y)
    np.testing.assert_allclose(tk.mahalanobis_sq(mean, cov, z), ref, rtol=1e-9)


def test_kalman_predict_closed_form_and_spd(rng):
    mean, cov = tk.kf_initiate(np.array([100.0, 50.0, 0.4, 120.0]))
    assert np.all(mean[4:] == 0) and np.all(np.diag(cov) > 0)
    for step in range(1000):
        m2, c2 = tk.kf_predict(mean, cov)
        np.testing.assert_array_equal(m2[:4], mean[:4] + mean[4:])
        np.testing.assert_array_equal(m2[4:], mean[4:])
        z = m2[:4] + rng.normal(0, 1, 4) * [3, 3, 0.01, 3]
        mean, cov = tk.kf_update(m2, c2, z)
        assert np.array_equal(cov, cov.T)
        np.linalg.cholesky(cov)                                   # raises if not SPD


def test_kalman_update_joseph_equals_simple_form(rng):
    """For the optimal gain the Joseph form equals (I - K H) P."""
    a = rng.standard_normal((8, 8))
    p = a @ a.T + np.eye(8)
    mean = np.array([5.0, 6.0, 0.5, 30.0, 1, 1, 0, 0])
    z = np.array([6.0, 5.0, 0.55, 31.0])
    m2, p2 = tk.kf_update(mean, p, z)
    r = tk.measurement_noise(mean)
    hm = tk.H_MAT
    s = hm @ p @ hm.T + r
    k = p @ hm.T @ np.linalg.inv(s)
    np.testing.assert_allclose(m2, mean + k @ (z - hm @ mean), rtol=1e-10)
    simple = (np.eye(8) - k @ hm) @ p
    np.testing.assert_allclose(p2, 0.5 * (simple + simple.T), rtol=1e-8, atol=1e-10)


def test_kalman_tracks_constant_velocity():
    truth = np.array([100.0, 200.0, 0.5, 80.0])
    vel = np.array([2.0, -1.0, 0.0, 0.5])
    mean, cov = tk.kf_initiate(truth)
    for t in range(1, 200):
        mean, cov = tk.kf_predict(mean, cov)
        mean, cov = tk.kf_update(mean, cov, truth + vel * t)
    np.testing.assert_allclose(mean[4:], vel, atol=1e-3)
    np.testing.assert_allclose(mean[:4], truth + vel * 199, atol=1e-2)


def _brute_assign(c, max_cost):
    t_n, d_n = c.shape
    best = None
    if t_n <= d_n:
        cands = ((list(range(t_n)), list(p)) for p in itertools.permutations(range(d_n), t_n))
    else:
        cands = ((list(p), list(range(d_n))) for p in itertools.permutations(range(t_n), d_n))
    for rows, cols in cands:
        vals = c[rows, cols]
        ok = vals <= max_cost
        key = (-int(ok.sum()), float(vals[ok].sum()))
        if best is None or key < best:
            best = key
    return -best[0], best[1]


@pytest.mark.parametrize("t_n,d_n", [(3, 3), (4, 6), (6, 4), (5, 5), (1, 4), (7, 7)])
def test_assign_matches_brute_force(rng, t_n, d_n):
    for _ in range(5):
        c = rng.uniform(0, 1.2, (t_n, d_n))
        c[rng.random((t_n, d_n)) < 0.3] = np.inf
        pairs, total = tk.assign(c, 0.7)
        n_ok, best = _brute_assign(c, 0.7)
        assert len(pairs) == n_ok
        assert total == pytest.approx(best, abs=1e-12)
        assert len(set(pairs[:, 0])) == len(pairs) and len(set(pairs[:, 1])) == len(pairs)
        assert np.all(c[pairs[:, 0], pairs[:, 1]] <= 0.7)


def test_assign_empty():
    pairs, total = tk.assign(np.zeros((0, 5)), 0.7)
    assert pairs.shape == (0, 2) and total == 0.0


def test_synthetic_cost_has_both_gated_and_open_pairs():
    s = synthetic_dets_tracks(5, 40, 40, 64)
    c = tk.cost_matrix(s["trk_emb"], s["mean"], s["cov"], s["boxes"], s["det_emb"])
    assert np.isinf(c).mean() > 0.5 and np.isfinite(c).sum() >= 20
    fin = c[np.isfinite(c)]
    assert fin.min() >= 0 and fin.max() <= 2


def test_tracker_keeps_identities_on_clean_synthetic_scene(rng):
    """Ground-truth rectangles with small noise and per-identity embeddings: each
    identity keeps one track id; a vanished object is removed after max_lost."""
    n = 6
    pos = rng.uniform(100, 500, (n, 2))
    vel = rng.uniform(-3, 3, (n, 2))
    size = np.stack([rng.uniform(20, 40, n), rng.uniform(60, 120, n)], 1)
    ident = rng.standard_normal((n, 32))
    ident /= np.linalg.norm(ident, axis=1, keepdims=True)
    trk = tk.Tracker(max_cost=0.7, max_lost=5)
    owner = {}
    for t in range(40):
        alive = range(n) if t < 20 else range(n - 1)              # object n-1 leaves at t = 20
        boxes, embs = [], []
        for i in alive:
            c = pos[i] + vel[i] * t + rng.normal(0, 0.5, 2)
            boxes.append([c[0] - size[i, 0] / 2, c[1] - size[i, 1] / 2, c[0] + size[i, 0] / 2, c[1] + size[i, 1] / 2])
            e = ident[i] + 0.05 * rng.standard_normal(32)
            embs.append(e / np.linalg.norm(e))
        order = rng.permutation(len(boxes))
        trk.step(np.array(boxes)[order], np.array(embs)[order])
        for tr in trk.tracks:
            if tr["lost"] == 0:
                i = int(np.argmax(ident @ tr["emb"]))
                owner.setdefault(i, tr["id"])
                assert owner[i] == tr["id"]
    assert len(owner) == n
    assert len(trk.tracks) == n - 1


def test_box_to_z_hand_computed():
    """(x1, y1, x2, y2) = (10, 20, 40, 110): centre (25, 65), width 30, height 90,
    so the aspect a = w / h = 1/3 (not h / w = 3)."""
    z = tk.box_to_z(np.array([[10.0, 20.0, 40.0, 110.0], [-5.0, 0.0, 15.0, 80.0]]))
    np.testing.assert_array_equal(z[0], [25.0, 65.0, 30.0 / 90.0, 90.0])
    np.testing.assert_array_equal(z[1], [5.0, 40.0, 0.25, 80.0])


def test_smooth_embedding_closed_form():
    """Orthogonal unit f (track) and e (detection): f' = (0.9 f + 0.1 e) / sqrt(0.82),
    so <f', f> = 0.9 / sqrt(0.82) and <f', e> = 0.1 / sqrt(0.82); the old state
    carries the momentum.  A scaled-up e does not change the direction of the
    weights beyond the stated mix (e enters unnormalised)."""
    f = np.zeros(16)
    f[3] = 1.0
    e = np.zeros(16)
    e[7] = 1.0
    g = tk.smooth_embedding(f, e)
    assert abs(np.linalg.norm(g) - 1.0) < 1e-15
    assert g @ f == pytest.approx(0.9 / math.sqrt(0.82), rel=1e-14)
    assert g @ e == pytest.approx(0.1 / math.sqrt(0.82), rel=1e-14)
    g2 = tk.smooth_embedding(f, 3.0 * e)
    assert g2 @ e / (g2 @ f) == pytest.approx(0.3 / 0.9, rel=1e-14)


def test_kalman_predict_covariance_closed_form():
    """P = diag(p), F = [[I, I], [0, I]]: F P F^T has P[i, i] = p_i + p_{i+4},
    P[i, i+4] = P[i+4, i] = p_{i+4}, P[i+4, i+4] = p_{i+4}; the process noise Q is
    added on the diagonal with stds scaled by the height before the prediction
    (position h/20, velocity h/160; a: 1e-2, va: 1e-5)."""
    p = np.arange(1.0, 9.0) * 0.37
    h = 120.0
    mean = np.array([300.0, 200.0, 0.4, h, 1.5, -2.0, 0.01, 6.0])     # vh != 0: h changes on predict
    m2, c2 = tk.kf_predict(mean, np.diag(p))
    q = np.array([(h / 20) ** 2, (h / 20) ** 2, 1e-4, (h / 20) ** 2,
                  (h / 160) ** 2, (h / 160) ** 2, 1e-10, (h / 160) ** 2])
    want = np.zeros((8, 8))
    for i in range(4):
        want[i, i] = p[i] + p[i + 4] + q[i]
        want[i, i + 4] = want[i + 4, i] = p[i + 4]
        want[i + 4, i + 4] = p[i + 4] + q[i + 4]
    np.testing.assert_allclose(c2, want, rtol=1e-14, atol=0)
    np.testing.assert_array_equal(m2, np.concatenate([mean[:4] + mean[4:], mean[4:]]))


def test_kalman_steady_state_matches_discrete_riccati():
    """With a constant height the filter splits into four independent 1-D
    constant-velocity filters with constant Q and R; after many predict/update
    steps the predicted 2x2 covariance of each coordinate is the solution of the
    discrete algebraic Riccati equation X = F X F^T - F X H^T (H X H^T + r)^-1 H X F^T + Q
    (scipy.linalg.solve_discrete_are with A = F^T, B = H^T)."""
    from scipy.linalg import solve_discrete_are
    h = 90.0
    z = np.array([200.0, 150.0, 0.35, h])
    mean, cov = tk.kf_initiate(z)
    for _ in range(400):
        mean, cov = tk.kf_predict(mean, cov)
        pred = cov.copy()
        mean, cov = tk.kf_update(mean, cov, z)
    assert mean[3] == h
    f1 = np.array([[1.0, 1.0], [0.0, 1.0]])
    h1 = np.array([[1.0], [0.0]])
    # cx, cy and h share the height-scaled noises (the aspect's 1e-10 velocity
    # noise makes its filter converge over thousands of steps, so it is left out)
    q = np.diag([(h / 20) ** 2, (h / 160) ** 2])
    x = solve_discrete_are(f1.T, h1, q, np.array([[(h / 20) ** 2]]))
    for i in (0, 1, 3):
        got = pred[np.ix_([i, i + 4], [i, i + 4])]
        np.testing.assert_allclose(got, x, rtol=1e-10)


def test_fused_cost_reduces_to_its_parts(rng):
    """Motion weight 0 is the appearance cost; weight 1 is the Mahalanobis
    distance itself where the gate passes; the gate pattern never changes."""
    from jde_inputs import synthetic_dets_tracks
    s = synthetic_dets_tracks(12, 20, 30, 64)
    args = (s["trk_emb"], s["mean"], s["cov"], s["boxes"], s["det_emb"])
    from oracle import track as otrack
    base = otrack.cost_matrix(*args)
    c0 = otrack.fused_cost_matrix(*args, 0.0)
    np.testing.assert_array_equal(np.isinf(c0), np.isinf(base))
    np.testing.assert_allclose(c0[np.isfinite(base)], base[np.isfinite(base)], rtol=0, atol=1e-15)
    c1 = otrack.fused_cost_matrix(*args, 1.0)
    d2 = otrack.gate_distances(s["mean"], s["cov"], s["boxes"])
    fin = np.isfinite(base)
    np.testing.assert_allclose(c1[fin], d2[fin], rtol=1e-15)
    cw = otrack.fused_cost_matrix(*args, 0.02)
    np.testing.assert_allclose(cw[fin], 0.98 * base[fin] + 0.02 * d2[fin], rtol=1e-14)


def test_iou_cost_closed_forms():
    from oracle import track as otrack
    # a track state (cx, cy, a, h) whose box is (0, 0, 2, 1): cx 1, cy 0.5, h 1, a 2
    m = np.array([[1.0, 0.5, 2.0, 1.0, 0, 0, 0, 0]])
    boxes = np.array([[0, 0, 2, 1], [1, 0, 3, 1], [5, 5, 6, 6], [0, 0, 1, 1]], dtype=np.float64)
    c = otrack.iou_cost_matrix(m, boxes)[0]
    np.testing.assert_allclose(c, [0.0, 1.0 - 1.0 / 3.0, 1.0, 1.0 - 0.5], atol=1e-15)
    np.testing.assert_allclose(otrack.state_to_box(m)[0], [0, 0, 2, 1])
