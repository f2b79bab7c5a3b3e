"""MI355X (gfx950) event-camera intensity reconstruction on the event manifold.

The compute path is the HIP library ``librec.so`` (C ABI in include/rec.h);
``paper_1607_06283_amd.rec`` is its ctypes binding.  Nothing here falls back
to CPU code: without the built library the binding raises.
"""
__all__ = ["rec", "build"]
