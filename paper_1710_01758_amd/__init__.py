"""MI355X-native PCG-in-Split-Bregman reconstruction with the circulant (BCCB)
preconditioner of Koolstra, van Gemert et al. (arXiv 1710.01758).

The compute path lives in the native library ``libpics.so`` (HIP kernels for
gfx950 behind a C ABI, declared in ``include/pics.h``).  ``binding`` marshals
arguments to it; ``inputs`` draws seeded synthetic workloads.  Importing this
package does not load the library; ``binding.lib()`` does, and raises if it
is missing.
"""
__all__ = ["inputs", "binding"]
