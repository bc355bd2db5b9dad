"""gfx950 (MI355X) library for linear regression estimation (LRE) of quantum states
from local Pauli measurement counts (arXiv:1602.08604: steps (i) and (ii), and the
step (iii) projection as a separate call).

The compute path is liblre.so (HIP); ``lre`` is its ctypes binding.
"""
from .lre import (LRE_NO_RHO, LRE_RHO_FP32, LRE_WHT_MFMA, LreError, check_flags,  # noqa: F401
                  estimate, pauli_sums, signed_sums, workspace_bytes)
