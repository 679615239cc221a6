"""MI355X (gfx950) batched silhouette fitness for CMA-ES instrument tracking.

The hot path (CMA-ES sample -> forward kinematics -> transform/project/snap ->
integer raster -> mask counts -> loss -> CMA-ES update) runs in the HIP
kernels of ``libtk.so`` behind the C ABI of ``include/tk.h``; ``tk`` is its
ctypes binding and ``tracker`` drives whole generations.
"""
from . import tk  # noqa: F401

__all__ = ["tk"]
