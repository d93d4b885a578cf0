"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Holds no arithmetic of the method itself: it only draws ensembles,
parameter fields and upstream gradients."""
from .synth import *  # noqa: F401,F403
