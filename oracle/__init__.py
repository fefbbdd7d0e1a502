"""CPU oracle for blocked LU with tournament pivoting.

Test infrastructure only: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.
"""
