"""Plain CPU oracle of the screen-space lattice-offset optimiser.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run this package; the product path
(the HIP library and its Python binding) never does.

Written from the paper (Belcour & Heitz, "Lessons Learned and Improvements
when Building Screen-Space Samplers with Blue-Noise Error Distribution",
SIGGRAPH 2021 Talks): Sec. 2 and Eq. (1) (energy and test integrands),
Sec. 3.2 (rank-1 lattice and toroidal scrambling), Sec. 3.3 (blur criterion),
Sec. 3.4 (parallel optimisation).  NumPy, FP64 for real values and exact
int64 for lattice indices and hit counts.  It shares no code with the HIP
path; the only common dependency is the seeded input generator ``synthgen``.

Parity status per function is recorded in each module and in the design
notes; every function here is pinned by a CPU test against values printed in
the paper, closed forms, invariants, brute force or an independent library
routine.
"""
from . import energy, estimator, integrands, lattice, philox, quality, sweep  # noqa: F401
