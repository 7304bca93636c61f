"""Plain FP64 CPU oracle for the constant-potential electrostatics path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the GPU library.

Every function is written from the definitions in Tee & Searles,
"Fully Periodic, Computationally Efficient Constant Potential Molecular
Dynamics Simulations of Ionic Liquid Supercapacitors" (arXiv 2201.12963),
in NumPy/SciPy double precision, without blocking or fusion beyond what the
definitions state, so that each step can be checked against the paper by eye.

Modules
-------
ewald   exact Ewald sums with Gaussian electrode charges (Eq. 1-3)
pppm    particle-particle particle-mesh sums with the same splitting
cpm     the electroneutral constant-potential solve (Eq. 4-15), energy,
        forces and the adjoint gradient
slab    the charged-sheet correction of the slab geometry (Fig. 2b)
cells   cell binning of electrolyte sites (integer reference)

Parity status: every function here is pinned by the CPU tests in
tests/test_oracle_*.py (closed forms, invariances, brute-force sums,
finite differences, textbook special cases).
"""

KE = 1.43996454784  # Coulomb constant 1/(4 pi eps0) in eV nm / e^2
