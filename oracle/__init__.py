"""Plain FP64 CPU reference of the method (test infrastructure only).

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The product path never does.
"""
