"""MI355X (gfx950) hot path of phaseless AFQMC with a stochastically sampled
correlated trial wave function.

The computation lives in libafqmc.so (HIP kernels behind the C ABI declared in
include/afqmc.h); ``paper_2505_18519_amd.afqmc`` is its ctypes binding and
``paper_2505_18519_amd.driver`` sequences one step.  Importing this package
loads nothing; the binding loads the library on first use and raises if it is
missing.
"""
