"""Unbiased Markov chain pool decoding on MI355X (gfx950).

``native`` is the ctypes binding of the C ABI (include/mcpd.h) implemented by
the in-tree HIP library ``libmcpd.so``; ``instances`` holds the seeded
synthetic workloads.  Importing the package loads nothing.
"""

__all__ = ["native", "instances", "build"]
