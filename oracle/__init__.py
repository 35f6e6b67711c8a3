"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 implementations of what the HIP path computes, written from the paper.
Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this package.
"""
