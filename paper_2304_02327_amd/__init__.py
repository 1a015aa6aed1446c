"""Direction-split ("phisplit") exponential integrators on AMD MI355X.

The computation lives in the C-ABI library ``libexpint.so`` (declared in
``include/expint.h``); this package is its Python binding.  Importing it
raises ImportError if the library has not been built.
"""

from ._binding import (  # noqa: F401
    C128,
    EXPORTED_SYMBOLS,
    F64,
    LIB_PATH,
    NOALLOC_SCRATCH_BYTES,
    NONLIN,
    PREC_BF16X3,
    PREC_FP32,
    PREC_FP64,
    PREC_SLICED,
    SCHEMES,
    ExpintError,
    Plan,
    RiccatiBatch,
    matrix_to_device,
    phi_setup,
    tensor_from_device,
    tensor_to_device,
    tucker_apply,
    tucker_apply_noalloc,
    tucker_workspace_size,
    tucker_fuses_modes12,
    tucker_tune,
    version,
)
