"""MI355X-native hybrid PIC/MCC discharge stepper (arXiv 1508.02892).

The hot path (field solve, ion fluid, electron push / null-collision Monte
Carlo / deposit, append, compaction + sort) runs in hand-written HIP kernels
for gfx950 behind the C ABI declared in ``include/hd.h``.  ``hd`` is a thin
ctypes binding of that ABI; ``workloads`` defines the seeded synthetic inputs.
Importing this package does not load the native library.
"""
__all__ = ["hd", "workloads"]
