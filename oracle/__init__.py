"""FP64 CPU oracle (test infrastructure only; never imported by the GPU product path)."""
from .gp_oracle import *  # noqa: F401,F403
from . import gp_adjoint  # noqa: F401
