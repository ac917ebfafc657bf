"""Seeded synthetic inputs for the JDE hot path.

This package is the only code shared by the HIP path and the FP64 oracle.  It
draws random numbers and lays out input structure (frame pixels, raw weights,
anchor sizes, synthetic tracks); it holds none of the method's arithmetic
(no convolution, decode, suppression, normalisation, cost or filtering).

The stand-ins replace what the paper measures on and is trained with: MOT16
FullHD sequences resized to 1088x608 (Sec. 5, Table 2) and trained JDE weights
(Sec. 3.1).  Neither is reproduced; the recipes are seeded and synthetic.
"""

from .configs import ModelConfig, TINY, FULL, SEED_BASE, model_config  # noqa: F401
from .frames import tiny_frame, scene_frame, scene_batch, scene_objects, capture_frame  # noqa: F401
from .weights import (weight_specs, raw_weights, model_weights, load_calib,  # noqa: F401
                      anchors_px, CALIB_DIR)
from .tracks import synthetic_dets_tracks  # noqa: F401
from .mixes import ragged_mix, mix_frames, MIX_SIZES  # noqa: F401
