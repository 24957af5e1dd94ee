"""PROPAGATE-P seed-bitset propagation on MI355X (gfx950).

The compute path is the HIP library ``libpp.so`` (sources in ``csrc/``,
C interface in ``include/pp.h``).  ``paper_2301_06499_amd.pp`` is the thin
ctypes binding with the same entry-point names; ``inputs`` holds the seeded
graph generators.  Importing the package does not load the library: the
binding loads it on first use and raises if it is missing.
"""
__all__ = ["inputs", "pp"]
