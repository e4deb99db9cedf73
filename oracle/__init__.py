"""CPU oracle for the extremum graph (test infrastructure only).

``oracle.oracle`` wraps the plain C implementation; ``oracle.brute`` is a
literal pure-Python version for tiny grids.  Neither may be used by the GPU
library: only tests, the smoke entry point and the benchmark's CPU-baseline
leg import this package.
"""
