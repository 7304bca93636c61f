"""Seeded synthetic inputs for the constant-potential electrostatics path.

This package only builds input data: cell sizes, electrode atom positions,
electrolyte site positions and charges, and the numerical parameters
(splitting parameter, cutoffs, mesh) each workload is run with.  It holds
none of the method's arithmetic.  Both the CPU oracle and the GPU path read
their inputs from here, so the two see identical arrays.

Workloads (lengths in nm, charges in e, potentials in V):

* ``tiny``       -- 1.476 x 1.27824 x 6.0 cell, two single-layer graphene
                    electrodes of 72 atoms, 50 + 50 single-site ions,
                    explicit Ewald k-space.
* ``paper``      -- 3.4 x 3.4 x 12.625 cell shaped after the paper's
                    supercapacitor (appendix, equilibration paragraph):
                    proximal graphene layers of 440 atoms, 320 coarse-grained
                    ion pairs, PPPM order 5.
* ``large``      -- 6.8 x 6.8 x 12.625 cell, 1760 atoms per proximal layer,
                    1280 ion pairs, PPPM order 5.

Each comes in finite-field (``ff``) and doubled-cell (``dc``) geometry.
"""

from .cells import (  # noqa: F401
    Workload,
    make_workload,
    perturbed_frames,
    random_walk,
    WORKLOAD_NAMES,
    MDSetup,
    md_setup,
)
