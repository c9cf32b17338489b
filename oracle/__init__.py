"""CPU oracle for cascade-hashing matching and the MBR block schedule.

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg import it; the product path never does.
"""
