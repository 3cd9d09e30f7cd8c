"""FP64 CPU oracle for the SMS-MUSSELS IRLS solve.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark; never by the GPU library.
"""
from .smsm_oracle import *  # noqa: F401,F403
from . import smsm_oracle  # noqa: F401
