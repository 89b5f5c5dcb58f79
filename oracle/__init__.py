"""FP64 CPU oracle for the octree MUSCL-Hancock / MinMod / HLLC hydro step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path
never does.  It shares no code with the GPU library.
"""
