"""MI355X-native odd-even Kalman smoother (Gargir & Toledo, IPDPS 2025).

The compute path is the HIP library ``libks.so`` (C ABI declared in
include/ks.h); ``paper_2502_11686_amd.ks`` is its Python binding.  Importing the
package loads nothing: the library is opened on first use, and every entry point
raises if it is missing -- there is no CPU fallback.
"""
__all__ = ["gen", "ks"]
