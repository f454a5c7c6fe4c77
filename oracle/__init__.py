"""Plain FP64 CPU oracle for column-generation direct aperture optimisation.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or
links this package: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library; the only
thing both sides take from a common module is the seeded input generator
(:mod:`phantom`), which holds none of the method's arithmetic.

Everything here is written for a reader checking it against the paper by eye:
NumPy / SciPy FP64 arrays, ``math.fsum`` for totals that decide things, and
pure-Python loops only where the paper's own description is a loop over a
handful of items (MLC rows, apertures).

Modules
-------
``model``     per-structure objective coefficients (eq. 9, eq. 10), dose
              d = D x (eq. 1, eq. 2 and eq. 7), objective F and its gradient
              (eq. 3 to eq. 5 in per-structure form), beamlet prices
              w = D^T grad F (the bracket of eq. 8).
``aperture``  aperture <-> beamlet maps: x = A y (eq. 7) and A^T g.
``pricing``   the pricing sub-problem (eq. 8, Section 2.3): min-sum leaf
              interval per MLC row by enumeration, per-beam sums, argmin.
``master``    the restricted master by gradient projection with an exact line
              search (Section 2.3; the step rule is this package's reading).
``solve``     the column-generation loop (Section 2.2, Section 2.3).
``metrics``   plan metrics: PTV D95 and organ-at-risk Dmax.

Parity pins
-----------
Each function is pinned in ``tests/`` by something other than itself
(closed forms, brute-force enumeration, SciPy solvers, invariants).  Only the
trajectory of a full multi-round solve beyond those invariants is
"parity unpinned": the paper prints no apertures, objective values or
iteration counts to compare against.
"""
from .model import (Problem, make_problem, voxel_coefficients, structure_sizes, reoptimization_structures,  # noqa: F401
                    dose, objective, grad_objective, prices)
from .aperture import Aperture, beamlet_intensity, aperture_gradient  # noqa: F401
from .pricing import price_row, price, ranked_apertures  # noqa: F401
from .master import line_search, MasterState, master_step, solve_master  # noqa: F401
from .solve import solve  # noqa: F401
from .metrics import d95, dmax  # noqa: F401
