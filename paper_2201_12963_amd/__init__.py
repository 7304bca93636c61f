"""MI355X-native constant-potential (CPM) electrostatics: HIP kernels behind a C-ABI.

Python side: `binding.Context` wraps the C-ABI library (libcpm.so, built by
`paper_2201_12963_amd.build`).  Importing the package does not touch the GPU.
"""

from .binding import (  # noqa: F401
    Context, CpmError, MDLoop, load_library,
    FINITE_FIELD, DOUBLED_CELL, SLAB, KSPACE_EWALD, KSPACE_PPPM, FP64, MIXED,
)
