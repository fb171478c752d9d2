"""CPU oracle of the convective right-hand side, the viscous fluxes and the
reaction source (test infrastructure only)."""
from .xf_oracle import *  # noqa: F401,F403
from . import xf_oracle  # noqa: F401
from . import xf_viscous  # noqa: F401
from . import xf_reaction  # noqa: F401
