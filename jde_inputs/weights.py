"""Seeded weights of the synthetic JDE networks, and the weight blob order.

Weight list order (the blob format both sides consume, one entry per conv):

  stem                              3x3, 3 -> c0
  s{1..5}.down                      3x3 stride 2, C -> 2C
  s{s}.b{i}.c1, s{s}.b{i}.c2        1x1 C -> C/2, then 3x3 C/2 -> C (residual block)
  for the heads at strides 32, 16, 8 (in that order), with F = C_level / 2:
    p{l}.set0 .. set4               1x1 Cin->F, 3x3 F->2F, 1x1 2F->F, 3x3 F->2F, 1x1 2F->F
    p{l}.det3                       3x3 F -> 2F
    p{l}.det1                       1x1 2F -> 6A   (linear output; channel 6a+k,
                                    k = dx, dy, dw, dh, c_bg, c_fg)
    p{l}.emb                        3x3 F -> E     (linear output)
    lat{l} (l = 32, 16 only)        1x1 F -> F/2   (feeds the next, finer level)

Each entry is (w [Cout, k, k, Cin], b [Cout]) in FP32.

Raw weights are He-normal (std sqrt(2 / (Cin k^2))) drawn in FP64 from
PCG64(seed, layer index).  A trained network would carry batch-norm layers;
the stand-in folds a batch norm (gamma 1, beta 0, eps 1e-5) whose statistics
are the per-channel mean and variance of each conv's pre-activation on a
calibration frame: w' = w / sqrt(var + eps), b' = -mean / sqrt(var + eps).
Those statistics, and the confidence offsets beta_K that put about K anchors
over the 0.5 threshold, come from the stored calibration file that the
oracle's calibration script writes; this module only applies them.  Box-delta
channels of the det outputs get gain 0.1 so decoded boxes stay near anchors.
"""

import os

import numpy as np

from .configs import ModelConfig

CALIB_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "calib")
BN_EPS = 1e-5
BOX_DELTA_GAIN = 0.1


def weight_specs(cfg: ModelConfig):
    """List of (name, cout, k, cin, kind); kind is 'bn', 'det' or 'emb'."""
    specs = []
    c = cfg.c0
    specs.append(("stem", c, 3, 3, "bn"))
    level_c = {}
    for s, nb in enumerate(cfg.blocks, 1):
        specs.append((f"s{s}.down", 2 * c, 3, c, "bn"))
        c *= 2
        for i in range(nb):
            specs.append((f"s{s}.b{i}.c1", c // 2, 1, c, "bn"))
            specs.append((f"s{s}.b{i}.c2", c, 3, c // 2, "bn"))
        level_c[s] = c
    nout = 6 * cfg.num_anchors
    lat = 0
    for lvl, stage in ((32, 5), (16, 4), (8, 3)):
        cin = level_c[stage] + lat
        f = level_c[stage] // 2
        specs += [
            (f"p{lvl}.set0", f, 1, cin, "bn"),
            (f"p{lvl}.set1", 2 * f, 3, f, "bn"),
            (f"p{lvl}.set2", f, 1, 2 * f, "bn"),
            (f"p{lvl}.set3", 2 * f, 3, f, "bn"),
            (f"p{lvl}.set4", f, 1, 2 * f, "bn"),
            (f"p{lvl}.det3", 2 * f, 3, f, "bn"),
            (f"p{lvl}.det1", nout, 1, 2 * f, "det"),
            (f"p{lvl}.emb", cfg.emb_dim, 3, f, "emb"),
        ]
        if lvl != 8:
            specs.append((f"lat{lvl}", f // 2, 1, f, "bn"))
            lat = f // 2
    return specs


def raw_weights(cfg: ModelConfig):
    """List of FP64 He-normal weight arrays [Cout, k, k, Cin], one per conv."""
    out = []
    for i, (name, cout, k, cin, kind) in enumerate(weight_specs(cfg)):
        r = np.random.Generator(np.random.PCG64([cfg.seed, 101, i]))
        w = r.standard_normal((cout, k, k, cin)) * np.sqrt(2.0 / (cin * k * k))
        if kind == "det":
            gain = np.ones(cout)
            for a in range(cout // 6):
                gain[6 * a:6 * a + 4] = BOX_DELTA_GAIN
            w = w * gain[:, None, None, None]
        out.append(w)
    return out


def anchors_px(cfg: ModelConfig):
    """[3, A, 2] anchor (w, h) in pixels for strides 8, 16, 32.

    12 pedestrian-shaped anchors (w:h = 1:3) with heights 24 * (640/24)^(k/11)
    at the 608-row frame, four per stride, scaled by the config's anchor scale.
    """
    a = cfg.num_anchors
    k = np.arange(3 * a)
    h = 24.0 * (640.0 / 24.0) ** (k / (3 * a - 1)) * cfg.anchor_scale
    wh = np.stack([h / 3.0, h], axis=-1)
    return wh.reshape(3, a, 2).astype(np.float32)


def load_calib(cfg: ModelConfig):
    """Stored calibration of ``cfg``: dict with 'mu', 'var' (per BN layer) and 'beta' (per K)."""
    path = os.path.join(CALIB_DIR, f"{cfg.name}.npz")
    if not os.path.exists(path):
        raise FileNotFoundError(f"calibration file {path} is missing; run oracle/make_calib.py")
    z = np.load(path, allow_pickle=False)
    specs = weight_specs(cfg)
    bn_idx = [i for i, s in enumerate(specs) if s[4] == "bn"]
    offs = z["bn_offsets"]
    mu = {i: z["mu"][offs[j]:offs[j + 1]] for j, i in enumerate(bn_idx)}
    var = {i: z["var"][offs[j]:offs[j + 1]] for j, i in enumerate(bn_idx)}
    beta = {int(k): float(b) for k, b in zip(z["beta_k"], z["beta"])}
    return {"mu": mu, "var": var, "beta": beta}


def fold_layers(cfg: ModelConfig, raw, mu, var, beta: float = 0.0):
    """Apply folded batch norm with the given statistics; FP32 (w, b) list.

    ``mu``/``var`` map BN-layer index -> per-channel FP64 statistics.  The
    confidence offset ``beta`` is added to every c_fg bias of the det outputs.
    """
    layers = []
    for i, (name, cout, k, cin, kind) in enumerate(weight_specs(cfg)):
        w = raw[i]
        if kind == "bn":
            s = 1.0 / np.sqrt(var[i] + BN_EPS)
            wf = w * s[:, None, None, None]
            b = -mu[i] * s
        else:
            wf = w
            b = np.zeros(cout)
            if kind == "det":
                b[5::6] = beta
        layers.append((wf.astype(np.float32), b.astype(np.float32)))
    return layers


def model_weights(cfg: ModelConfig, k_candidates=None, calib=None):
    """FP32 (w, b) list for ``cfg``; ``k_candidates`` selects the stored beta_K (None: beta 0)."""
    calib = load_calib(cfg) if calib is None else calib
    beta = 0.0 if k_candidates is None else calib["beta"][int(k_candidates)]
    return fold_layers(cfg, raw_weights(cfg), calib["mu"], calib["var"], beta)
