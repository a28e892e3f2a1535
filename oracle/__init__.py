"""CPU reference of the per-frame bisection update (test infrastructure).

Only the test-suite, the entry point's smoke check and the benchmark's CPU
baseline load this package.  It wraps ``libcbt_oracle.so`` (plain C, built by
``oracle.build.build()``) with ctypes and shares no code with the HIP library.
"""
from .oracle import Oracle, OracleError, Stats, cbt_reduce, one_to_bit, zero_to_bit, load  # noqa: F401
