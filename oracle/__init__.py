"""FP64 CPU oracle (test infrastructure only; never imported by the product path)."""
from .ptycho_oracle import *  # noqa: F401,F403
from .ptycho_oracle import __all__  # noqa: F401
