"""FermiNet VMC hot path on MI355X (gfx950).

The compute path is the HIP library ``libferminet.so`` behind the C ABI
declared in ``include/ferminet.h``; ``paper_2011_07125_amd.ferminet`` is
its thin ctypes binding.  Importing this package loads nothing; the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["inputs", "ferminet"]
