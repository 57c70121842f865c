"""CPU oracle (test infrastructure only; see shen_oracle's module docstring)."""
from .shen_oracle import *  # noqa: F401,F403
from . import shen_oracle  # noqa: F401
