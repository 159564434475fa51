"""FP64 CPU oracle (test infrastructure only; never imported by the product path)."""
from . import pty_oracle, toy  # noqa: F401
