"""FP64 CPU oracles of SMS-MUSSELS: the IRLS solve (smsm_oracle), the
augmented-Lagrangian solve (al_oracle) and the learned unrolled solver
(learned_oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark; never by the GPU library.
"""
from .smsm_oracle import *  # noqa: F401,F403
from . import smsm_oracle  # noqa: F401
