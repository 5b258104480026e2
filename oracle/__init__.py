"""CPU FP64 oracle for the eigenvector-eigenvalue identity (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import anything from this package.  The GPU library never links, imports or
calls it, and the two share no code; only the seeded input generators serve
both.
"""
from .eeid_oracle import *  # noqa: F401,F403
from .eeid_oracle import FLAG_DEGENERATE, FLAG_NONFINITE_INPUT  # noqa: F401
