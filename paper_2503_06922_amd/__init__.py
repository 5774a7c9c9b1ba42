"""MI355X (gfx950) contact-FEM hot path: co-rotational beam Newton loop with lumen contacts.

The computation lives in the HIP library ``libaccfem.so`` (C ABI in
include/accfem.h); ``paper_2503_06922_amd.fem`` is its ctypes binding and ``paper_2503_06922_amd.autograd`` the
torch.autograd wrapper (FEMEquilibrium) around its solve and adjoint.
"""
from .fem import (Context, FemError, params_from_batch, state_to_PR, lib,  # noqa: F401
                  FEM_FP64, FEM_MIXED, FEM_ACT_CABLES, FEM_ACT_TIP_WRENCH_LOCAL,
                  FEM_ACT_TIP_WRENCH_GLOBAL, FEM_ACT_CABLE_WRENCH)

