"""CPU oracle for the WCSPH step -- test infrastructure only.

Only the test-suite, the package's smoke check and the benchmark's CPU
baseline leg may import this package.  The product path (the HIP library and
its binding) never imports, links or calls it.
"""
