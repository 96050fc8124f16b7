"""FP64 CPU oracle of the destriping hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never does, and this package never
imports the library.
"""
