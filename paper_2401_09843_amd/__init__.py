"""MI355X spectral hyperviscosity Navier-Stokes solver (arXiv:2401.09843).

The solver itself lives in the HIP library libns.so (C ABI: include/ns.h);
`paper_2401_09843_amd.ns` is its thin ctypes binding.  Importing this package
does not load the library.
"""
__all__ = ["ns", "inputs"]
