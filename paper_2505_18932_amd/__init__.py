"""MI355X (gfx950) geometry stage of online multi-view video synthesis
(arXiv 2505.18932): z-buffered pixel-Gaussian splatting, frustum-volume TSDF
fusion with a running temporal weight, zero-crossing extraction, colour-
difference masks with the temporally filtered depth, the volume-free
raymarch, EWA front-to-back compositing, the blending network's input maps
and blend, adjoints and a batched path, as hand-written HIP kernels behind a
C ABI (include/ggeom.h).
"""
from . import _lib, autograd
from .ops import (BatchPlan, blend_views, camera, cameras, difference_masks, mask_params,
                  network_inputs,
                  relative_projection, splat_params, splat_views,
                  splat_views_backward, splat_views_ewa, timing_enable, timing_read, timing_reset,
                  tsdf_extract_depth, tsdf_extract_depth_backward, tsdf_integrate,
                  tsdf_integrate_backward, tsdf_integrate_noalloc, tsdf_params, tsdf_raymarch,
                  tsdf_view_table, volume_tuning,
                  workspace_size)

__all__ = ["BatchPlan", "blend_views", "camera", "cameras", "difference_masks", "mask_params",
           "network_inputs",
           "relative_projection", "splat_params", "splat_views",
           "splat_views_backward", "splat_views_ewa", "timing_enable", "timing_read", "timing_reset",
           "tsdf_extract_depth", "tsdf_extract_depth_backward", "tsdf_integrate",
           "tsdf_integrate_backward", "tsdf_integrate_noalloc", "tsdf_params", "tsdf_raymarch",
           "tsdf_view_table", "volume_tuning",
           "workspace_size", "_lib",
           "autograd"]
