"""CPU FP64 oracle of the periodic RPA hot path (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this package; the library never does.
"""
