"""FP64 CPU oracle for the dual-k-mesh TDA-BSE hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product
path (the HIP library and its Python binding) never calls it and shares
no code with it.

Everything here is plain numpy in float64/complex128, written from the
paper's equations in the paper's order, without blocking or fusion:

* Fourier interpolation of W_munu(R) to W_munu(q) (Sec. III.B, dual-k-mesh
  workflow; phase convention of Eq. (W_LRI));
* LRI pair densities in the Kohn-Sham basis (Sec. III.A, the definition
  of C-tilde);
* the explicit Tamm-Dancoff Hamiltonian A (Eq. (Hamiltonian) with the
  kernel integrals of Eq. (W_LRI) and its exchange companion);
* its diagonalisation and the velocity-form absorption spectrum
  (Eq. (abs_vel)) with Lorentzian broadening;
* an independent Haydock/Lanczos recurrence with full re-orthogonalisation
  and its continued fraction (not in the paper: Haydock, Heine & Kelly
  1972; Benedict & Shirley 1999);
* gradients of Re<Ybar, H X>, of the lowest exciton energy
  (Hellmann-Feynman) and of the spectrum (exact resolvent).

Parity pins (tests/test_oracle_*.py) tie every function to something other
than itself: closed forms, invariants, brute force on tiny inputs and
library routines.  Functions whose constants have no such pin are marked
"parity unpinned" in their docstrings.
"""
from .bse_ref import *  # noqa: F401,F403
