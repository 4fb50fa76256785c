"""Plain FP64 CPU oracle for POLFED (polynomially filtered exact diagonalization).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the GPU library.

Every function here is written to be checked against the paper by eye: no
blocking, fusion or reordering beyond what the cited formula states.  Library
primitives (scipy sparse mat-vec, numpy dense eigensolvers, ARPACK Lanczos for
the spectral extremes) serve as single steps.

Modules
  basis    sector enumeration and ranks (ascending-integer order)
  models   random-field XXZ chain, quantum sun, spinless t-V fermions as CSR
  filter   Chebyshev delta filter, Clenshaw evaluation, Gaussian DOS, order K
  lanczos  spectral bounds, filtered Lanczos with full reorthogonalization,
           eigenpair extraction
  polfed   the full workflow (Sec. 4.6 of the paper)
  dense    dense diagonalization reference for small systems
"""
from . import basis, models, filter, lanczos, polfed, dense  # noqa: F401
