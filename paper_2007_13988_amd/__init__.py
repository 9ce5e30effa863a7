"""MI355X (gfx950) hierarchical surface localization and mesh-free rendering for a
pixel-aligned implicit function.  The compute path is libpifu.so (HIP); this package
holds its build script and the ctypes binding."""
from .pifu import (FIELD_ELLIPSOIDS, FIELD_MLP, FIELD_PLANE, AsyncBatchedGrid,  # noqa: F401
                   AsyncGrid, AsyncRender,
                   BatchedGrid,
                   DeviceField, DeviceMLP, GridOutputs, RenderOutputs, autotune, autotune_clear,
                   convert, eval_points, fp8_calibrate, grid_opts, load_library, occupancy_grid,
                   occupancy_grid_into, profile_enable, profile_read, render_opts, render_view,
                   render_view_into, render_view_traced, grid_and_render_into, octree_grid,
                   octree_grid_into, mesh)
