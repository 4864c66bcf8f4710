"""FP64 CPU oracle of the PRIEST projection and sampling loop (test infrastructure only).

Only tests, the package smoke check and the benchmark's CPU-baseline leg may
import this package; the product path never does.
"""
from .priest_oracle import *  # noqa: F401,F403
