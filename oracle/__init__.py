"""Plain CPU oracle for multiple-precision dense C := AB.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the GPU library and its binding never do.
"""
