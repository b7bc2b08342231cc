"""CPU oracle for the FCIQMC iteration (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this package; the product library never imports it.
"""
