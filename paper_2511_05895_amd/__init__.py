"""Exact maximum flow / minimum cut on AMD MI355X (gfx950) with dynamic capacity
updates: push-relabel after Kannappan, Kumar and Nasre (arXiv 2511.05895).

The library is libmf.so (C-ABI in include/mf.h); ``paper_2511_05895_amd.mf``
is its thin ctypes binding.  Import of ``mf`` fails loudly when the library
is not built: there is no CPU fallback."""

__all__ = ["mf"]
