"""MI355X (gfx950) scanline DP and extended DP with the recursive minimum search.

Mozerov, "Extended Dynamic Programming and Fast Multidimensional Search
Algorithm for Energy Minimization in Stereo and Motion", arXiv 1410.7922.
The solvers live in ``libedp.so`` (C ABI: include/edp.h); ``binding`` marshals
torch tensors into it.
"""
from .binding import (  # noqa: F401
    EDP_E_TIMEOUT, PRIOR_LINEAR, PRIOR_SQUARED, TRUNC_JOINT, TRUNC_PER_DIM, BatchPlan, EdpError, Workspace,
    check_status, dp_marginals, dp_scanline, dsi, energy, load, solve, solve_windowed, tile_depth, tile_info, tiles,
    tiles_3d, wide_tiles, wide_tiles_3d, workspace_size)
