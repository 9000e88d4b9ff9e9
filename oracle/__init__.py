"""CPU oracle for DDPS -- test infrastructure only.

Imported by the tests, the package's smoke check and the benchmark's CPU
baseline leg; never by the GPU path.  Plain float64 numpy/scipy.
"""
