"""FP64 CPU oracle for the implicit FLD radiation step.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.
"""
from .fld_oracle import *  # noqa: F401,F403
