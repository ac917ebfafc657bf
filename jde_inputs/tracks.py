"""Seeded synthetic detections and tracks for the tracks x detections cost.

Detections are pedestrian-shaped boxes (height U[40, 300] px, aspect
U[0.3, 0.6]) placed uniformly in the frame, with embeddings drawn uniformly on
the unit sphere.  A fraction of the tracks sits near a detection (the same
box in measurement space plus noise, an embedding close to the detection's);
the rest are unrelated.  Track covariances are random symmetric positive
definite matrices with height-scaled standard deviations.
"""

import numpy as np


def _unit_rows(r, n, e):
    v = r.standard_normal((n, e))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def synthetic_dets_tracks(seed: int, T: int, D: int, E: int, height: int = 608,
                          width: int = 1088, frac_near: float = 0.7):
    """Return a dict of FP32 det boxes [D,4] (x1,y1,x2,y2), det emb [D,E],
    track emb [T,E], FP64 track mean [T,8] = (cx, cy, a, h, vcx, vcy, va, vh)
    and FP64 track cov [T,8,8]."""
    r = np.random.Generator(np.random.PCG64([seed, 17, T, D, E]))
    h = r.uniform(40.0, 300.0, D) * height / 608.0
    a = r.uniform(0.3, 0.6, D)
    cx = r.uniform(0.0, width, D)
    cy = r.uniform(0.0, height, D)
    w = a * h
    boxes = np.stack([cx - w / 2, cy - h / 2, cx + w / 2, cy + h / 2], axis=1).astype(np.float32)
    det_emb = _unit_rows(r, D, E).astype(np.float32)

    mean = np.zeros((T, 8))
    trk_emb = _unit_rows(r, T, E)
    n_near = min(int(round(frac_near * min(T, D))), T, D)
    near = r.permutation(D)[:n_near]
    for t in range(T):
        if t < n_near:
            d = near[t]
            mean[t, :4] = (cx[d], cy[d], a[d], h[d])
            mean[t, :4] += r.normal(0.0, 1.0, 4) * (0.03 * h[d], 0.03 * h[d], 0.01, 0.03 * h[d])
            v = det_emb[d] + 0.3 * r.standard_normal(E) / np.sqrt(E)
            trk_emb[t] = v / np.linalg.norm(v)
        else:
            th = r.uniform(40.0, 300.0) * height / 608.0
            mean[t, :4] = (r.uniform(0, width), r.uniform(0, height), r.uniform(0.3, 0.6), th)
        mean[t, 4:] = r.normal(0.0, 1.0, 4) * (2.0, 2.0, 1e-3, 0.5)
    cov = np.zeros((T, 8, 8))
    for t in range(T):
        hh = mean[t, 3]
        std = np.array([hh / 10, hh / 10, 2e-2, hh / 10, hh / 16, hh / 16, 1e-4, hh / 16])
        A = np.eye(8) + 0.3 * r.standard_normal((8, 8))
        C = A @ A.T / 8.0 + 0.5 * np.eye(8)
        cov[t] = std[:, None] * C * std[None, :]
        cov[t] = 0.5 * (cov[t] + cov[t].T)
    return {"boxes": boxes, "det_emb": det_emb, "trk_emb": trk_emb.astype(np.float32),
            "mean": mean, "cov": cov}
