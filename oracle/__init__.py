"""CPU oracle of the convective right-hand side (test infrastructure only)."""
from .xf_oracle import *  # noqa: F401,F403
from . import xf_oracle  # noqa: F401
