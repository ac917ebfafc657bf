"""Model configurations of the two synthetic JDE networks.

Both follow the paper's description of the model (Sec. 3.1): a Darknet-53
style backbone, an FPN that upsamples higher levels and fuses them with lower
ones, and prediction heads at three strides.  The trained network is not
available, so these are random-weight stand-ins with the same shapes.
"""

from dataclasses import dataclass
from typing import Tuple

# Frame t of stream s under seed S is a pure function of (S, s, t).
SEED_BASE = 2011039100


@dataclass(frozen=True)
class ModelConfig:
    name: str
    c0: int                      # stem width; stage s has c0 * 2**s channels
    blocks: Tuple[int, ...]      # residual blocks per stage (5 stages)
    emb_dim: int                 # appearance embedding length (512 in the paper's output row)
    num_anchors: int             # anchors per cell per scale
    height: int                  # native input height (divisible by 32)
    width: int                   # native input width (divisible by 32)
    anchor_scale: float          # anchor sizes relative to the 608-row frame

    @property
    def seed(self) -> int:
        return SEED_BASE + (0 if self.name == "tiny" else 1)


# 3x192x320, c0 = 16, blocks 1/1/2/2/1, 64-d embeddings.
TINY = ModelConfig("tiny", 16, (1, 1, 2, 2, 1), 64, 4, 192, 320, 192.0 / 608.0)
# Darknet-53 widths 32..1024 with blocks 1/2/8/8/4, 512-d embeddings, 3x608x1088.
FULL = ModelConfig("full", 32, (1, 2, 8, 8, 4), 512, 4, 608, 1088, 1.0)

_BY_NAME = {"tiny": TINY, "full": FULL}


def model_config(name: str) -> ModelConfig:
    return _BY_NAME[name]
