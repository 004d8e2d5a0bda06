"""MI355X-native Strang-split fiber monodomain solver.

The compute path is the C-ABI library ``libfib.so`` (HIP kernels for gfx950)
declared in ``include/fib.h``; ``paper_2107_07104_amd.fib`` is its thin
ctypes binding.  ``paper_2107_07104_amd.inputs`` builds seeded synthetic
workloads.  Importing the package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
