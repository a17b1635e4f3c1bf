"""FP64 CPU oracle for the photon-field hot path.

Test infrastructure only: the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may use it; the product path never does.
"""
