"""mvgs: multi-view differentiable Gaussian-splatting rasterizer for MI355X (gfx950).

The rasterizer itself is libmvgs.so (HIP kernels behind the C ABI of include/mvgs.h);
`_lib` binds it with ctypes and `raster` exposes it to PyTorch. `scenes` draws the seeded
synthetic inputs.
"""
from . import scenes  # noqa: F401

__all__ = ["scenes"]
