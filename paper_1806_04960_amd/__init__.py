"""MI355X-native explicit step of the well-balanced Osher-Romberg scheme for the reduced
Baer-Nunziato free-surface model (arXiv:1806.04960).

The compute path is the HIP library ``libbn2d.so`` (C ABI declared in ``include/bn2d.h``);
``paper_1806_04960_amd.bn2d`` is its ctypes binding.  ``scenarios`` builds seeded inputs.
"""
