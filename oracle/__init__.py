"""FP64 CPU oracle of ASKIT: test infrastructure only.

Imported by the tests, the smoke check and the benchmark's CPU-baseline
leg; never by the HIP library or its binding.
"""
