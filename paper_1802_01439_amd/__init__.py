"""dgmf: matrix-free DG operators (SIPG Laplace, convective LLF, its VJP, CG) for MI355X.

The compute path is the HIP library ``libdgmf.so`` (built by
``__graft_entry__.build()``) behind the C ABI declared in ``include/dgmf.h``;
``paper_1802_01439_amd.dgmf`` is its thin ctypes binding and
``paper_1802_01439_amd.autograd`` wraps the operators as torch autograd
functions.  Importing this package does not load the library.
"""
__version__ = "0.1.0"
