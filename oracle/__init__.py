"""FP64 CPU oracle for ConeGaussian rendering.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's CPU
baseline may use this package; the product path (the HIP library and its binding)
never imports it.  See ``conegauss_oracle.cpp`` for the definitions followed.
"""
from .oracle import *  # noqa: F401,F403
