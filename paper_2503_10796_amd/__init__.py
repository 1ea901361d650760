"""MI355X-native spherical-agent mechanics (uniform-grid neighbour search,
sphere-sphere forces, capped displacement, static-agent skip, growth and
division), batched parameter sweeps and a BF16-MFMA surrogate MLP.

The compute path is the HIP library ``libabm.so`` behind the C ABI declared
in ``include/abm.h``; ``paper_2503_10796_amd.abm`` is its ctypes binding.
Importing this package does not load the library; ``abm`` does, and fails
loudly when it is missing.
"""
