"""MI355X-native Saturating Coordinate Descent (SaCD) for sparse nonnegative
CP tensor factorization.

The GPU path lives in the C-ABI library ``libsacd.so`` (HIP kernels for
gfx950); ``paper_2003_03572_amd.sacd`` is its thin ctypes binding and
``paper_2003_03572_amd.gen`` draws seeded synthetic inputs.  Importing the
package loads nothing; the binding loads the library on first use and raises
if it is missing.
"""
__all__ = ["gen", "sacd"]
