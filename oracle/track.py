"""FP64 oracle of the association side: cost matrix, Kalman filter, assignment.

Test infrastructure only.  Follows Appendix A items 4-9: predict track
locations with a Kalman filter; cosine distance between detection embeddings
and the embeddings of active or lost tracks; pairs whose detection is too far
from the track's predicted location get infinite cost; Hungarian assignment;
pairs above a cost threshold are rejected; matched tracks are updated and
marked active, unmatched tracks become lost, and tracks lost for longer than a
threshold are removed.

Readings where the paper is silent:

* state (cx, cy, a, h, vcx, vcy, va, vh), a = w / h; constant velocity
  F = [[I, I], [0, I]], H = [I, 0];
* noise stds scale with the height: process pos h/20, vel h/160 (a: 1e-2 and
  1e-5); measurement h/20 for cx, cy, h and 1e-1 for a; initial 2x pos and 10x
  vel stds;
* "too far" is the squared Mahalanobis distance of the 4-d measurement under
  S = H P H^T + R, gated at the chi-square 95% quantile for 4 dof, 9.4877;
* cosine distance 1 - <f, e> clamped to [0, 2];
* assignment minimises total cost over complete matchings of size min(T, D)
  with entries above ``max_cost`` (and +inf) replaced by a constant larger
  than any feasible total, i.e. most feasible pairs first, then least cost;
  matched pairs above ``max_cost`` are then rejected;
* track embedding smoothing f <- normalise(0.9 f + 0.1 e);
* all tracks that are active or lost are predicted and appear as cost rows.
"""

import numpy as np
from scipy.optimize import linear_sum_assignment

STD_POS = 1.0 / 20.0
STD_VEL = 1.0 / 160.0
CHI2_4_95 = 9.4877
MOMENTUM = 0.9
NORM_EPS = 1e-12

F_MAT = np.block([[np.eye(4), np.eye(4)], [np.zeros((4, 4)), np.eye(4)]])
H_MAT = np.hstack([np.eye(4), np.zeros((4, 4))])


def box_to_z(box):
    """(x1, y1, x2, y2) -> measurement (cx, cy, a = w/h, h), FP64."""
    b = np.asarray(box, dtype=np.float64)
    w = b[..., 2] - b[..., 0]
    h = b[..., 3] - b[..., 1]
    return np.stack([(b[..., 0] + b[..., 2]) / 2.0, (b[..., 1] + b[..., 3]) / 2.0, w / h, h], axis=-1)


def kf_initiate(z):
    z = np.asarray(z, dtype=np.float64)
    h = z[3]
    mean = np.concatenate([z, np.zeros(4)])
    std = np.array([2 * STD_POS * h, 2 * STD_POS * h, 1e-2, 2 * STD_POS * h,
                    10 * STD_VEL * h, 10 * STD_VEL * h, 1e-5, 10 * STD_VEL * h])
    return mean, np.diag(std ** 2)


def process_noise(mean):
    h = mean[3]
    std = np.array([STD_POS * h, STD_POS * h, 1e-2, STD_POS * h,
                    STD_VEL * h, STD_VEL * h, 1e-5, STD_VEL * h])
    return np.diag(std ** 2)


def measurement_noise(mean):
    h = mean[3]
    std = np.array([STD_POS * h, STD_POS * h, 1e-1, STD_POS * h])
    return np.diag(std ** 2)


def kf_predict(mean, cov):
    """x <- F x; P <- F P F^T + Q (Q from the pre-predict height)."""
    q = process_noise(mean)
    return F_MAT @ mean, F_MAT @ cov @ F_MAT.T + q


def kf_project(mean, cov):
    """(H x, S = H P H^T + R)."""
    return H_MAT @ mean, H_MAT @ cov @ H_MAT.T + measurement_noise(mean)


def kf_update(mean, cov, z):
    """Textbook update with the Joseph-form covariance, then symmetrised."""
    r = measurement_noise(mean)
    hx, s = kf_project(mean, cov)
    k = np.linalg.solve(s, H_MAT @ cov).T          # K = P H^T S^-1 (S, P symmetric)
    y = np.asarray(z, dtype=np.float64) - hx
    mean2 = mean + k @ y
    ikh = np.eye(8) - k @ H_MAT
    cov2 = ikh @ cov @ ikh.T + k @ r @ k.T
    return mean2, 0.5 * (cov2 + cov2.T)


def mahalanobis_sq(mean, cov, zs):
    """Squared Mahalanobis distance of each measurement in zs [D, 4] to the track."""
    hx, s = kf_project(mean, cov)
    y = np.asarray(zs, dtype=np.float64).reshape(-1, 4) - hx
    sol = np.linalg.solve(s, y.T)
    return (y.T * sol).sum(axis=0)


def cost_matrix(trk_emb, mean, cov, det_boxes, det_emb, gate=CHI2_4_95):
    """C[t, d] = clamp(1 - <f_t, e_d>, 0, 2), or +inf when d^2_M(t, d) > gate.  FP64."""
    f = np.asarray(trk_emb, dtype=np.float64)
    e = np.asarray(det_emb, dtype=np.float64)
    c = np.clip(1.0 - f @ e.T, 0.0, 2.0)
    zs = box_to_z(np.asarray(det_boxes).reshape(-1, 4))
    for t in range(len(f)):
        d2 = mahalanobis_sq(mean[t], cov[t], zs)
        c[t, d2 > gate] = np.inf
    return c


def gate_distances(mean, cov, det_boxes):
    """[T, D] squared Mahalanobis distances (for reporting margins to the gate)."""
    zs = box_to_z(np.asarray(det_boxes).reshape(-1, 4))
    return np.stack([mahalanobis_sq(mean[t], cov[t], zs) for t in range(len(mean))]) \
        if len(mean) else np.zeros((0, len(zs)))


def fused_cost_matrix(trk_emb, mean, cov, det_boxes, det_emb, motion_weight, gate=CHI2_4_95):
    """Appearance and motion in one cost (an association variant beyond the
    paper's appendix): C = (1 - w) cos + w d^2_M where the gate passes, +inf where
    d^2_M > gate; w = 0 is the appearance-only cost of ``cost_matrix``.  FP64."""
    w = float(motion_weight)
    f = np.asarray(trk_emb, dtype=np.float64)
    e = np.asarray(det_emb, dtype=np.float64)
    cos = np.clip(1.0 - f @ e.T, 0.0, 2.0)
    zs = box_to_z(np.asarray(det_boxes).reshape(-1, 4))
    c = np.zeros_like(cos)
    for t in range(len(f)):
        d2 = mahalanobis_sq(mean[t], cov[t], zs)
        c[t] = (1.0 - w) * cos[t] + w * d2
        c[t, d2 > gate] = np.inf
    return c


def state_to_box(mean):
    """Kalman state (cx, cy, a, h, ...) -> box (x1, y1, x2, y2) with w = a h."""
    m = np.asarray(mean, dtype=np.float64)
    w = m[..., 2] * m[..., 3]
    h = m[..., 3]
    return np.stack([m[..., 0] - w / 2, m[..., 1] - h / 2, m[..., 0] + w / 2, m[..., 1] + h / 2], axis=-1)


def iou_cost_matrix(mean, det_boxes):
    """Second association stage on box overlap: C[t, d] = 1 - IoU(predicted box of
    track t, detection d), FP64 (1 for disjoint or empty boxes)."""
    a = state_to_box(np.asarray(mean).reshape(-1, 8))[:, None, :]
    b = np.asarray(det_boxes, dtype=np.float64).reshape(-1, 4)[None, :, :]
    iw = np.clip(np.minimum(a[..., 2], b[..., 2]) - np.maximum(a[..., 0], b[..., 0]), 0, None)
    ih = np.clip(np.minimum(a[..., 3], b[..., 3]) - np.maximum(a[..., 1], b[..., 1]), 0, None)
    inter = iw * ih
    uni = (a[..., 2] - a[..., 0]) * (a[..., 3] - a[..., 1]) + (b[..., 2] - b[..., 0]) * (b[..., 3] - b[..., 1]) - inter
    iou = np.where(uni > 0, inter / np.where(uni > 0, uni, 1.0), 0.0)
    return 1.0 - iou


def assign(cost, max_cost):
    """Min-cost assignment, then rejection of pairs above max_cost.

    Returns (pairs [P, 2] of (t, d) sorted by t, total cost of the kept pairs).
    """
    c = np.asarray(cost, dtype=np.float64)
    t_n, d_n = c.shape
    if t_n == 0 or d_n == 0:
        return np.zeros((0, 2), dtype=np.int64), 0.0
    big = 4.0 * (min(t_n, d_n) + 1) * max(2.0, float(max_cost)) + 1.0
    cm = np.where(c > max_cost, big, c)
    rows, cols = linear_sum_assignment(cm)
    ok = c[rows, cols] <= max_cost
    pairs = np.stack([rows[ok], cols[ok]], axis=1).astype(np.int64)
    return pairs, float(c[rows[ok], cols[ok]].sum())


def smooth_embedding(f, e):
    """f <- normalise(0.9 f + 0.1 e)."""
    v = MOMENTUM * np.asarray(f, dtype=np.float64) + (1.0 - MOMENTUM) * np.asarray(e, dtype=np.float64)
    return v / max(np.sqrt((v * v).sum()), NORM_EPS)


class Tracker:
    """Track lifecycle of Appendix A items 4-9 (FP64)."""

    def __init__(self, max_cost=0.7, max_lost=30, gate=CHI2_4_95):
        self.max_cost = max_cost
        self.max_lost = max_lost
        self.gate = gate
        self.tracks = []          # dicts: id, mean, cov, emb, lost (frames lost, 0 = active)
        self.next_id = 1

    def step(self, boxes, embs):
        boxes = np.asarray(boxes, dtype=np.float64).reshape(-1, 4)
        embs = np.asarray(embs, dtype=np.float64)
        for tr in self.tracks:
            tr["mean"], tr["cov"] = kf_predict(tr["mean"], tr["cov"])
        if self.tracks and len(boxes):
            c = cost_matrix(np.stack([t["emb"] for t in self.tracks]),
                            np.stack([t["mean"] for t in self.tracks]),
                            np.stack([t["cov"] for t in self.tracks]), boxes, embs, self.gate)
            pairs, _ = assign(c, self.max_cost)
        else:
            pairs = np.zeros((0, 2), dtype=np.int64)
        matched_t = set(int(t) for t in pairs[:, 0])
        matched_d = set(int(d) for d in pairs[:, 1])
        zs = box_to_z(boxes) if len(boxes) else np.zeros((0, 4))
        for t, d in pairs:
            tr = self.tracks[t]
            tr["mean"], tr["cov"] = kf_update(tr["mean"], tr["cov"], zs[d])
            tr["emb"] = smooth_embedding(tr["emb"], embs[d])
            tr["lost"] = 0
        survivors = []
        for i, tr in enumerate(self.tracks):
            if i not in matched_t:
                tr["lost"] += 1
                if tr["lost"] > self.max_lost:
                    continue
            survivors.append(tr)
        for d in range(len(boxes)):
            if d not in matched_d:
                m, p = kf_initiate(zs[d])
                survivors.append({"id": self.next_id, "mean": m, "cov": p,
                                  "emb": embs[d] / max(np.linalg.norm(embs[d]), NORM_EPS), "lost": 0})
                self.next_id += 1
        self.tracks = survivors
        return pairs
