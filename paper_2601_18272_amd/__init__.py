"""MI355X (gfx950) library for the lattice kinetic scheme with a passively moving rigid
body and its discrete adjoint (arXiv 2601.18272): Python binding of liblks_hip.so."""
from . import _lib  # noqa: F401
from .api import (LKSFunction, LksError, Buffers, adjoint, body_step, checkpoint_bytes,  # noqa: F401
                  forward, map_design, problem_struct, state_elems, workspace_bytes,
                  design_filter, design_filter_adjoint, filter_struct, filter_workspace_bytes,
                  cyclic_sector_points, design_cyclic_expand, design_cyclic_collect, mma_update,
                  mma_workspace_bytes, optimize, volume_constraint, coupling, adjoint_paper)
