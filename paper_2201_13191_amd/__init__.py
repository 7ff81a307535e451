"""MI355X-native Monte Carlo photon-transport forward projector (arXiv 2201.13191).

The product is the C-ABI library libmcx.so (HIP kernels for gfx950 plus the
host runtime, declared in include/mcx.h); `paper_2201_13191_amd.mcx` is its
thin ctypes binding and `paper_2201_13191_amd.inputs` builds synthetic inputs.
"""
