"""FP64 CPU oracle of the SEPSO planner hot path.

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never imports it.
"""
