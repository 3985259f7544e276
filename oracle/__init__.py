"""FP64 CPU oracle for the tactile FEM hot path (test infrastructure only).

This package is the reference the GPU library is checked against.  It is
plain numpy/scipy in float64, written from the paper's equations and
algorithms, and shares no code with the library.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never calls it.

Modules (each function cites the passage it follows):
  surface   Alg. 1 (surface extraction): surface triangles, parent tets, contact-face
            labels, candidates, rest vertex areas, lumped mass
  material  Eq. 1 (Lame), Eq. 2 (first Piola stress), Eq. 3/4 (Cauchy stress),
            the energy density whose derivative is Eq. 2, its Hessian and
            PSD projection
  fem       per-tet deformation gradient, elastic energy/gradient/Hessian
  contact   IPC log barrier and the analytic indenter signed distances
  stepper   the incremental potential of one implicit step (Sec. III-B) and
            its Newton minimiser
  extract   Eq. 4 per tet, Alg. 1 traction decomposition, Alg. 2 contact path

Every function here has at least one pin in tests/ against values the
mathematics fixes (closed forms, finite differences, invariants, brute force).
"""
from . import surface, material, fem, contact, stepper, extract  # noqa: F401
