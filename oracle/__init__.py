"""FP64 CPU oracle for the explicit as-S_N time step.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import anything from this package.  It shares no code,
tables or constants with the HIP library and imports nothing from it.
"""
