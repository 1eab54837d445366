"""MI355X-native Cahn-Hilliard ADI hot path (arXiv 2101.06550).

The compute path is the C-ABI library ``libchx.so`` (HIP kernels for gfx950);
``paper_2101_06550_amd.chx`` is its thin ctypes binding.  Importing this
package loads nothing: the binding loads the library on first use and raises
if it is missing (there is no CPU fallback).
"""
__all__ = ["chx", "inputs"]
