"""CPU oracle (test infrastructure only; see ``sps_oracle``)."""
from .sps_oracle import *  # noqa: F401,F403
from .sps_oracle import K_MAD, BLOCK_STRIDE, CAND_DTYPE  # noqa: F401
from . import cluster_oracle  # noqa: F401
from . import dedisp_oracle  # noqa: F401
from . import rfi_oracle  # noqa: F401
