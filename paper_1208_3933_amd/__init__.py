"""MI355X (gfx950) pool-parallel bounding for permutation flow-shop branch-and-bound.

The library (libfspbb.so, C ABI declared in include/fspbb.h) computes the
two-machine (Johnson / Lageweg-Lenstra-Rinnooy Kan) lower bound over pools of
sub-problems with hand-written HIP kernels, after Melab et al., "A
GPU-accelerated Branch-and-Bound Algorithm for the Flow-Shop Scheduling
Problem".  ``paper_1208_3933_amd.fspbb`` is the thin ctypes binding; it raises
if the HIP library has not been built.  ``paper_1208_3933_amd.gen`` holds the
seeded synthetic inputs.
"""
