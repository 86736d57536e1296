"""MI355X (gfx950) library for projective affine body dynamics.

The simulation runs in the HIP library libpabd.so (include/pabd.h); this
package holds its ctypes binding, the seeded scene generators, the serving loop
and the build script.
"""
from . import scenes  # noqa: F401
from ._lib import (Batch, Busy, Diverged, PabdError, Scene, device_count,  # noqa: F401
                   hbm_copy_probe, lib, scene_bytes, tune_cache_clear, tune_cache_size,
                   use_torch_allocator)
