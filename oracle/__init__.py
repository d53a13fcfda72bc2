"""Plain FP64 CPU oracle of the adaptive-precision EAM-ACE force evaluation.

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP library: only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it.  The
library never calls into it and shares no code, tables or constants with it; the two
meet only through the seeded inputs of the ``synth`` package.

Every function follows the paper (Immel, Drautz, Sutmann, "Adaptive-precision
potentials for large-scale atomistic simulations", arXiv:2411.03002) and states the
passage it implements.  Arithmetic is float64 throughout; the geometric decisions that
must match the library bit for bit (squared distances, centro-symmetry sums, switching
polynomials) are written with an explicit evaluation order and no fused operations.
Forces are the negative gradient of the written-out energy, taken by PyTorch autograd
on CPU float64 tensors.

Convention: ``w`` is the weight of the precise potential (ACE).  The paper's switching
parameter is the weight of the fast potential, lambda = 1 - w (Sec. II A, eq. energy_hyb).
"""

from . import geometry, precision, eam, ace, hybrid, verlet, mlp  # noqa: F401
