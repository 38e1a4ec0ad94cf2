"""MI355X (gfx950) random sequential adsorption of linear k-mers on a torus,
run to jamming with first-wrap (percolation) tracking -- arXiv:1810.06800.

The compute path is the HIP library ``librsa_hip.so`` behind the C ABI of
``include/rsa.h``; :mod:`paper_1810_06800_amd.rsa` is a thin ctypes binding
with the same names.  Importing this package loads nothing; the binding loads
the library on first use and raises if it is missing.
"""

__all__ = ["rsa", "workloads", "build"]
