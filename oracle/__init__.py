"""FP64 CPU oracle for SL1M (test infrastructure only; see sl1m_oracle)."""
from .sl1m_oracle import *  # noqa: F401,F403
from . import quadtree  # noqa: F401  (adaptive refinement, reading R17)
from . import coarse  # noqa: F401  (coarse-to-fine warm start, reading R18)
