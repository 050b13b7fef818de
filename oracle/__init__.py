"""Plain FP64 CPU oracle for NGF + curvature registration (test infrastructure).

This package is the independent definition against which the GPU path is
checked.  It is deliberately slow and literal: every quantity is computed in
float64 with numpy, in the order the paper's definitions state, without
blocking, fusion or reordering beyond what a definition itself permits.

Only the test suite, the smoke check of the entry module and the benchmark's
CPU-baseline leg may import it.  The product path (the HIP library and its
Python binding) never imports, calls or falls back to anything here, and this
package imports nothing from the product path: the two share only the seeded
input generator, which holds none of the method's arithmetic.

Model (Sec. 2.1, Eq. 1): J(y) = D(R, T(P y)) + alpha * S(y), where y lives on
a nodal deformation grid, P converts it to the cell-centred image grid, D is
the normalised-gradient-field distance of Eq. 2 and S the curvature
regulariser.  Readings of points the paper leaves open are stated in each
module and collected in the design notes.

Pinning status: every function here is pinned by a test in ``tests/`` against
something other than itself (closed forms, library routines, invariants,
finite differences or brute force); none is "parity unpinned".
"""

from .grids import (  # noqa: F401
    image_coords_1d, node_spacing, node_coords_1d, identity, index_map,
    index_map_f32, omega_sets, apply_P, apply_PT, downsample, pyramid, prolongate,
    level_shapes,
)
from .ngf import (  # noqa: F401
    warp, warp_T_adjoint, cdiff, cdiff_adj, ngf_terms, ngf_dgT,
)
from .regulariser import laplacian, curvature  # noqa: F401
from .objective import Problem, eval_J_grad, eval_J_grad_T  # noqa: F401
from .lbfgs import LBFGS, register, early_stop_met, INFO  # noqa: F401
