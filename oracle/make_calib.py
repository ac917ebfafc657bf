"""Write the stored calibration of the synthetic JDE networks (test infrastructure).

Calls only the oracle and the seeded input generators.  For each model config:

1. batch-norm statistics: the FP64 oracle runs the raw He-normal network on
   calibration frame 0 and records each BN conv's per-channel pre-activation
   mean and variance (oracle.network.calibrate_bn);
2. confidence offsets: with the folded FP32 weights and zero c_fg bias, the
   FP64 forward of the same frame gives every anchor's margin m = c_fg - c_bg;
   beta_K = -(m_(K) + m_(K+1)) / 2, with m_(k) the k-th largest margin, puts
   exactly K anchors at score >= 0.5 on that frame with the threshold mid-gap.

Usage: python -m oracle.make_calib [tiny|full ...]
Output: jde_inputs/calib/<name>.npz (allow_pickle=False).
"""

import os
import sys
import time

import numpy as np

from jde_inputs import TINY, FULL, weight_specs, raw_weights, tiny_frame, scene_frame, CALIB_DIR
from jde_inputs.weights import fold_layers
from oracle.network import calibrate_bn, forward

K_LISTS = {"tiny": (50,), "full": (10, 20, 40, 50, 100, 200, 1000)}


def calibration_frame(cfg):
    if cfg.name == "tiny":
        return tiny_frame(cfg.seed, 0, cfg.height, cfg.width)
    return scene_frame(cfg.seed, 0, 0, cfg.height, cfg.width)


def all_margins(out):
    ms = []
    for d in out["det"]:
        v = d[0].reshape(-1, 6)
        ms.append(v[:, 5] - v[:, 4])
    return np.concatenate(ms)


def make(cfg):
    t0 = time.time()
    frame = calibration_frame(cfg)[None]
    specs = weight_specs(cfg)
    kinds = [s[4] for s in specs]
    raw = raw_weights(cfg)
    mu, var = calibrate_bn(frame, raw, cfg.blocks, kinds)
    layers = fold_layers(cfg, raw, mu, var, 0.0)
    out = forward(frame, layers, cfg.blocks)
    m = np.sort(all_margins(out))[::-1]
    ks = np.array(K_LISTS[cfg.name], dtype=np.int64)
    beta = np.array([-(m[k - 1] + m[k]) / 2.0 for k in ks])
    bn_idx = [i for i, k in enumerate(kinds) if k == "bn"]
    offs = np.cumsum([0] + [len(mu[i]) for i in bn_idx]).astype(np.int64)
    os.makedirs(CALIB_DIR, exist_ok=True)
    path = os.path.join(CALIB_DIR, f"{cfg.name}.npz")
    np.savez(path, bn_offsets=offs, mu=np.concatenate([mu[i] for i in bn_idx]),
             var=np.concatenate([var[i] for i in bn_idx]), beta_k=ks, beta=beta)
    print(f"{cfg.name}: wrote {path} ({time.time() - t0:.1f} s); beta={dict(zip(ks.tolist(), beta.round(4).tolist()))}")


if __name__ == "__main__":
    names = sys.argv[1:] or ["tiny", "full"]
    for n in names:
        make({"tiny": TINY, "full": FULL}[n])
