"""paper_2505_18764_amd -- MI355X-native differentiable Gaussian-splat rasterizer.

The compute path is the HIP library ``libgsr.so`` (C ABI in ``include/gsr.h``); this package
binds it (``_lib``) and wraps it for PyTorch (``render``). Importing the package does not load
the library; the first call does, and fails loudly if it is not built.
"""
from ._lib import GsrError, gs_version  # noqa: F401
from .render import (GaussianRasterizeFn, Projected, Raster2DFn, RasterConfig,  # noqa: F401
                     Workspace, prepare_2d, project, project_backward, raster_backward,
                     raster_forward, rasterize_2d, rasterize_gaussians, sort_)

__all__ = ["GsrError", "gs_version", "GaussianRasterizeFn", "Raster2DFn", "RasterConfig",
           "Workspace", "Projected", "project", "prepare_2d", "sort_", "raster_forward",
           "raster_backward", "project_backward", "rasterize_gaussians", "rasterize_2d"]
