"""MI355X implementation of the periodized Coulomb sum of Gumerov & Duraiswami,
"A method to compute periodic sums" (arXiv:1310.4374).

The hot path -- near-set build, check-point sums, least-squares
coefficients, zero-mean constant, near pair sums and far-field expansion --
runs in hand-written HIP kernels behind the C ABI of include/periodic_sum.h.
This package only marshals torch tensors (device memory, streams) into it.
"""
from ._lib import (PS_FP32_ACC64, PS_FP64, PS_MEAN_NONE, PS_MEAN_ZERO, PeriodicSumError,  # noqa: F401
                   lib)
from .api import BatchedPlan, PeriodicEnergy, Plan, select_parameters  # noqa: F401
