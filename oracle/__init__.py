"""CPU oracle for the complex DD/QD Newton corrector.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg.  The product path never imports it.
"""
