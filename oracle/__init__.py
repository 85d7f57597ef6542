"""FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  It wraps ``liboracle.so`` (plain C, built from
``oracle.c`` by ``build_oracle``) with ctypes and shares no code with the
GPU library.
"""
from .pyoracle import (OracleMesh, build_oracle, oracle_lib, norms, area_sum, thomas,  # noqa: F401
                       tracer_vertical_column)
