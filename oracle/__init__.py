"""CPU FP64 oracle for the per-increment elasto-plastic solve.

Test infrastructure only: tests, the smoke check and the benchmark's CPU
baseline may use it.  The GPU library never imports, links or calls it.
"""
