"""FP64 CPU oracle (test infrastructure only; see ``fzp_oracle``)."""
from .fzp_oracle import *  # noqa: F401,F403
