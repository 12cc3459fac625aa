"""Plain FP64 CPU oracle for the mixed virtual element saddle-point solve.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package.
The product path (the HIP library and its Python binding) never calls it.

It follows the paper step by step and in its notation: scaled monomials and
the face/cell geometry (Section 2), the degrees of freedom, the divergence and
the L2 projector computed through integration by parts (Section 4.1), the
stabilised local forms (Section 4.3), the global saddle-point system
(Section 5), and the paper's two block-diagonal preconditioners inside a
right-preconditioned flexible GMRES (Section 5, eqs. B_D, block_schur,
block_diag).  It shares no code with the HIP library; the only common input
is the seeded generator module paper_1901_02330_amd.inputs.
"""

from .quadrature import tet_rule, tri_rule  # noqa: F401
from .geometry import face_geometry, cell_geometry  # noqa: F401
from .assemble import discretize  # noqa: F401
from .solvers import direct_solve, fgmres, block_schur, block_reg  # noqa: F401
