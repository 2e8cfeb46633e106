"""MI355X (gfx950) tile-local depth-binned 3D Gaussian splatting rasterizer.

The compute path is the HIP library ``libtilegs.so`` behind the C ABI in
``include/tilegs.h``; this package only marshals arguments to it.
"""
from ._lib import (ORDER_BINNED, ORDER_GLOBAL, RASTER_PLAIN, RASTER_WAVE, REPAIR_ALL, REPAIR_NONE,  # noqa: F401
                   REPAIR_RULES, TileGSError, LIB_PATH, EXPORTS, lib)
from .api import (BatchRenderer, Binned, Params, Renderer, camera_struct, paper_params, project,  # noqa: F401
                  project_backward, project_views, render, render_differentiable, to_device)
