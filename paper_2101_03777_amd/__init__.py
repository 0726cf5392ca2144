"""crhyb: hybridised Crouzeix-Raviart Stokes / Navier-Stokes solver for AMD MI355X (gfx950).

The solver is the HIP library libcrhyb.so (C ABI in include/crhyb.h); this
package is its thin Python binding.  Importing the package does not load the
library; load() does, and raises if it has not been built.
"""
from ._binding import (  # noqa: F401
    CR_BICGSTAB, CR_FP32_IR, Batch, CR_FP64, CR_NATURAL, CR_NS_NEWTON, CR_OP_ASSEMBLED, CR_OP_AUTO, CR_OP_ELEMENT,
    CR_PCG, CR_PC_COARSE, CR_PC_DEFAULT, CR_PC_JACOBI, CR_RCM, CR_STOKES, CRError, EXPORTS,
    LIB_PATH, Prepared, System, TorchAllocator, load, topology,
)
