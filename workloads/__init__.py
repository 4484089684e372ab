"""Seeded synthetic inputs shared by the HIP path's tests/benchmarks and the
oracle's tests.  Input generation only: nothing here evaluates an integral or
a J/K contraction."""
from .generators import *  # noqa: F401,F403
