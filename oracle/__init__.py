"""FP64 CPU oracle (test infrastructure only; see reference.py and
forward_model.py).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package. The GPU product path never imports or calls it.
"""
from .reference import *  # noqa: F401,F403
from . import reference, quality, forward_model  # noqa: F401
