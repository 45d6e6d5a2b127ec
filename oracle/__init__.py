"""FP64 CPU oracle and spectral tools.  TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
import this package; the HIP product path never does.
"""
