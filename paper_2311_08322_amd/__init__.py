"""MI355X-native stencil hot path: horizontal diffusion, implicit vertical
advection, their fused time step and adjoints, as HIP kernels for gfx950
behind a C ABI (``include/stencil.h``).

The HIP library is loaded lazily on first use; every entry point raises if
it is missing -- there is no CPU fallback.
"""
__all__ = ["inputs"]
