"""Device-side association (Kalman predict / update and the min-cost
assignment on the GPU) against the host FP64 library code and the oracle.

The device kernels take the host code's operations in the same order with no
contraction, so states must be bit-identical to the host's and the assignment
the same; against the oracle (textbook matrices, scipy's assignment) the states
agree to FP64 rounding and the assigned totals to 1e-9.
"""

import sys

import numpy as np
import pytest

from jde_inputs import synthetic_dets_tracks
from oracle import track as otrack

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible MI355X"
    return t


def _states(seed, T):
    s = synthetic_dets_tracks(seed, T, 1, 64)
    return np.ascontiguousarray(s["mean"]), np.ascontiguousarray(s["cov"])


def test_kf_predict_dev_equals_host_and_oracle(torch):
    from paper_2011_03910_amd import jde_kf_predict, jde_kf_predict_dev
    _say("case: kf predict dev T=1000")
    mean, cov = _states(5, 1000)
    hm, hc = mean.copy(), cov.copy()
    jde_kf_predict(hm, hc)
    dm, dc = torch.from_numpy(mean.copy()).cuda(), torch.from_numpy(cov.copy()).cuda()
    jde_kf_predict_dev(dm, dc)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dm.cpu().numpy(), hm)
    np.testing.assert_array_equal(dc.cpu().numpy(), hc)
    for t in (0, 17, 999):
        om, oc = otrack.kf_predict(mean[t], cov[t])
        np.testing.assert_allclose(hm[t], om, rtol=1e-13, atol=1e-12)
        np.testing.assert_allclose(hc[t], oc, rtol=1e-12, atol=1e-12)
    jde_kf_predict_dev(dm[:0], dc[:0])          # T = 0 is a no-op


def test_kf_update_dev_equals_host_and_oracle(torch):
    """Three frames of tracks; each track takes the box of its assigned detection
    (or none); the device update equals the host jde_kf_update_n bitwise."""
    from paper_2011_03910_amd import jde_kf_update_dev, jde_kf_update_n, jde_box_to_z
    _say("case: kf update dev, 3 frames")
    cap = 64
    Ts = [30, 0, 45]
    tb = np.concatenate([[0], np.cumsum(Ts)]).astype(np.int32)
    mean, cov = _states(9, int(tb[-1]))
    rng = np.random.Generator(np.random.PCG64(31))
    boxes = np.zeros((3 * cap, 4), dtype=np.float32)
    d_of_t = np.full(int(tb[-1]), -1, dtype=np.int32)
    for f in range(3):
        s = synthetic_dets_tracks(40 + f, max(Ts[f], 1), cap, 64)
        boxes[f * cap:(f + 1) * cap] = s["boxes"]
        for t in range(tb[f], tb[f + 1]):
            if rng.random() < 0.7:
                d_of_t[t] = rng.integers(cap)
    hm, hc = mean.copy(), cov.copy()
    ti = np.nonzero(d_of_t >= 0)[0]
    f_of_t = np.searchsorted(tb, ti, side="right") - 1
    z = jde_box_to_z(boxes)
    jde_kf_update_n(ti, f_of_t * cap + d_of_t[ti], hm, hc, z)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dm, dc = cu(mean), cu(cov)
    status = torch.full((int(tb[-1]),), -5, dtype=torch.int32, device="cuda")
    jde_kf_update_dev(tb, cu(d_of_t), {"boxes": cu(boxes), "count": cu(np.array(Ts, np.int32))}, cap, dm, dc, status)
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == 0).all()
    np.testing.assert_array_equal(dm.cpu().numpy(), hm)
    np.testing.assert_array_equal(dc.cpu().numpy(), hc)
    for t in ti[:5]:
        f = f_of_t[list(ti).index(t)]
        om, oc = otrack.kf_update(mean[t], cov[t], otrack.box_to_z(boxes[f * cap + d_of_t[t]].astype(np.float64)))
        np.testing.assert_allclose(hm[t], om, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(hc[t], oc, rtol=1e-8, atol=1e-9)


def _cost(rng, T, D, forbid=0.3):
    c = rng.uniform(0.0, 1.2, (T, D)).astype(np.float32)
    c[rng.random((T, D)) < forbid] = np.inf
    return c


@pytest.mark.parametrize("shapes", [
    [(40, 50), (0, 5), (7, 0), (1, 1), (200, 200)],
    [(300, 120), (120, 300), (64, 64)],
    [(1000, 1000)],
    [(2048, 700)],
])
def test_assign_dev_equals_host_and_oracle(torch, shapes):
    """Batched device assignment (one workgroup per frame) against the host
    Hungarian (same pairs) and scipy's assignment total on the allowed entries."""
    from paper_2011_03910_amd import jde_assign, jde_assign_dev
    _say(f"case: assign dev {shapes}")
    rng = np.random.Generator(np.random.PCG64(sum(t * 7 + d for t, d in shapes)))
    max_cost = 0.7
    cap = max(max(d for _, d in shapes), 1)
    cap = (cap + 63) // 64 * 64
    Ts = [t for t, _ in shapes]
    tb = np.concatenate([[0], np.cumsum(Ts)]).astype(np.int32)
    big = np.full((max(int(tb[-1]), 1), cap), -3.0, dtype=np.float32)
    costs = []
    for f, (T, D) in enumerate(shapes):
        c = _cost(rng, T, D)
        costs.append(c)
        big[tb[f]:tb[f + 1], :D] = c
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    counts = cu(np.array([d for _, d in shapes], np.int32))
    out = jde_assign_dev(cu(big), tb, {"count": counts}, cap, max_cost)
    torch.cuda.synchronize()
    dot = out["det_of_track"].cpu().numpy()
    tod = out["track_of_det"].cpu().numpy().reshape(len(shapes), cap)
    kept = out["kept"].cpu().numpy()
    total = out["total"].cpu().numpy()
    assert (out["status"].cpu().numpy() == 0).all()
    for f, (T, D) in enumerate(shapes):
        pairs, htotal = jde_assign(costs[f], max_cost)
        hd = np.full(T, -1)
        if len(pairs):
            hd[pairs[:, 0]] = pairs[:, 1]
        np.testing.assert_array_equal(dot[tb[f]:tb[f + 1]], hd)
        assert kept[f] == len(pairs)
        assert abs(total[f] - htotal) <= 1e-12 * max(1.0, abs(htotal))
        ht = np.full(D, -1)
        if len(pairs):
            ht[pairs[:, 1]] = pairs[:, 0]
        np.testing.assert_array_equal(tod[f, :D], ht)
        if T and D:
            ref, ref_total = otrack.assign(costs[f].astype(np.float64), max_cost)
            assert len(ref) == kept[f] and abs(ref_total - total[f]) <= 1e-9 * max(1.0, abs(ref_total))
        _say(f"  frame {f} {T}x{D}: kept {kept[f]} total {total[f]:.6f}")


def _batched_inputs(torch, shapes, E=512, seed=3):
    cap = 64 * ((max(max(d for _, d in shapes), 1) + 63) // 64)
    Ts = [t for t, _ in shapes]
    tb = np.concatenate([[0], np.cumsum(Ts)]).astype(np.int32)
    syn = [synthetic_dets_tracks(seed + f, max(T, 1), max(D, 1), E) for f, (T, D) in enumerate(shapes)]
    cat = lambda k: np.concatenate([s[k][:T] for s, (T, _) in zip(syn, shapes)])
    boxes = np.zeros((len(shapes) * cap, 4), np.float32)
    emb = np.zeros((len(shapes) * cap, E), np.float32)
    for f, (s, (T, D)) in enumerate(zip(syn, shapes)):
        boxes[f * cap:f * cap + D] = s["boxes"][:D]
        emb[f * cap:f * cap + D] = s["det_emb"][:D]
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dets = {"boxes": cu(boxes), "emb": cu(emb), "count": cu(np.array([d for _, d in shapes], np.int32))}
    return syn, tb, cap, cat, dets, cu


@pytest.mark.parametrize("w", [0.0, 0.02, 1.0])
def test_fused_cost_batch_vs_oracle(torch, w):
    from paper_2011_03910_amd import jde_cost_matrix_batch_fused
    shapes = [(33, 97), (0, 5), (40, 1), (64, 64)]
    _say(f"case: fused cost w={w} {shapes}")
    syn, tb, cap, cat, dets, cu = _batched_inputs(torch, shapes)
    got = jde_cost_matrix_batch_fused(cu(cat("trk_emb")), cu(cat("mean")), cu(cat("cov")), tb, dets, cap, w)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    for f, (s, (T, D)) in enumerate(zip(syn, shapes)):
        if not (T and D):
            continue
        ref = otrack.fused_cost_matrix(s["trk_emb"][:T], s["mean"][:T], s["cov"][:T], s["boxes"][:D],
                                       s["det_emb"][:D], w)
        g = got[tb[f]:tb[f + 1], :D]
        d2 = otrack.gate_distances(s["mean"][:T], s["cov"][:T], s["boxes"][:D])
        clear = np.abs(d2 - otrack.CHI2_4_95) > 1e-9 * otrack.CHI2_4_95
        np.testing.assert_array_equal(np.isinf(g)[clear], np.isinf(ref)[clear])
        fin = np.isfinite(ref) & np.isfinite(g)
        err = np.abs(g[fin] - ref[fin]) / np.maximum(1.0, np.abs(ref[fin]))
        assert err.max(initial=0) <= 2e-6, err.max()


def test_iou_cost_batch_vs_oracle(torch):
    from paper_2011_03910_amd import jde_iou_cost_batch
    shapes = [(33, 97), (7, 0), (50, 50)]
    _say(f"case: iou cost {shapes}")
    syn, tb, cap, cat, dets, cu = _batched_inputs(torch, shapes, seed=8)
    got = jde_iou_cost_batch(cu(cat("mean")), tb, dets, cap).cpu().numpy()
    n_overlap = 0
    for f, (s, (T, D)) in enumerate(zip(syn, shapes)):
        if not (T and D):
            continue
        ref = otrack.iou_cost_matrix(s["mean"][:T], s["boxes"][:D])
        g = got[tb[f]:tb[f + 1], :D]
        np.testing.assert_allclose(g, ref, rtol=0, atol=1e-6)
        n_overlap += int((ref < 1).sum())
        assert np.isnan(got[tb[f]:tb[f + 1], D:]).all()
    assert n_overlap > 0
