"""FP64 CPU oracle of spherical-agent mechanics and of the surrogate MLP.

Test infrastructure only: the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library.
"""
