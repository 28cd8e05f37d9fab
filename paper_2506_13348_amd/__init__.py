"""texsplat on MI355X: tile-based rendering of textured planar Gaussians (TextureSplat,
arXiv 2506.13348) with hand-written gfx950 HIP kernels behind a C ABI (include/texsplat.h).

Python here only marshals arguments: `_ffi` mirrors the C entry points one to one, `render`
keeps scenes and buffers on the device and enqueues the kernels."""
from . import _ffi
from ._ffi import lib
from .render import BatchRaster, DeviceScene, EnvTables, RenderPlan, cameras_tensor, render

__all__ = ["BatchRaster", "DeviceScene", "EnvTables", "RenderPlan", "cameras_tensor", "render", "lib", "_ffi"]
