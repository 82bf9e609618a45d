"""MI355X (gfx950) BFV multiply+relinearize and the p=17 modular-to-bit bridge.

The compute path is the C-ABI shared library built from ``csrc/`` (HIP kernels
for gfx950); ``fhe`` is its thin ctypes binding.  ``inputs`` holds the seeded
synthetic draws and parameter sets.
"""
