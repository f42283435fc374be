"""MI355X (gfx950) balanced 3DGS tile rasterizer: HIP kernels behind the C ABI
in include/bgs.h (libbgs.so), with a thin torch binding.

    from paper_2412_17378_amd import Rasterizer, make_cfg, render
"""
from .bgs import BgsError, lib, make_cfg  # noqa: F401
from .pipeline import Prepared, Rasterizer, Render3DFn, RenderFn, render, render_gaussians  # noqa: F401
