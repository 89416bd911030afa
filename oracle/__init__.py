"""Plain FP64 CPU oracle for the stochastic fermion-loop path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, the smoke check and the benchmark's CPU
baseline do.  It shares no code with the HIP implementation: the two are
independent derivations of the same mathematics, compared on the same seeded
inputs (which come from the separate ``synth`` module).

What it computes (paper: "A QUDA-branch to compute disconnected diagrams in
GPUs", LATTICE 2013):

* the stochastic inversions ``M s_r = eta_r`` of Section 2, eq. (1), for the
  twisted-mass Wilson operator, with Z2 / Z4 volume noise (Sections 2, 2.3, 2.4);
* the truncated solver method of Section 2.1: many low-precision solves plus a
  few high-precision corrections;
* the one-end-trick loops of Section 2.1.1 / 2.2: ultra-local and
  one-derivative insertions, with and without tau_3, built from the colour-
  traced 4x4 Dirac outer product and projected to momenta up to a p^2 cut.

The paper does not write down the operator, the gamma basis, the estimator
identities, the derivative stencil or the Fourier sign; each reading taken
here is stated in the docstring of the function that uses it.

Modules
-------
dirac   gamma matrices, lattice geometry, the operator, its even-odd Schur form
noise   SplitMix64 counter generator and Z2 / Z4 volume sources
solver  even-odd CGNR (same algorithm as the GPU path) and exact dense solves
loops   one-end-trick contractions, insertions, momentum projection, TSM
grad    adjoint-solve gradients of the loops with respect to eta and mu
hpe     hopping parameter expansion of the loops without tau_3
dilution  time-diluted sources and their single-slice estimators
clover  the clover term of the operator (Section 2.4's Wilson-and-clover variant)
"""
from . import dirac, noise, solver, loops  # noqa: F401
