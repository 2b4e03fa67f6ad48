"""Oracle for the matrix-free P1 (and 2D P2) operators: test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP path.
"""
