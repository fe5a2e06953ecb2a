"""Plain FP64 CPU oracle for HSWO / HSEG / RHSEG.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package. The GPU library
never calls it, and the two share no code: the only thing they have in common
is the seeded input generator module, which holds no segmentation arithmetic.

The C++ implementation (``hswo_oracle.cpp``) follows Section 4.1 of the paper
(the HSEG steps, the RHSEG recursion, Equation 1); see the header comment
there for the readings taken where the paper is silent.
"""
from .oracle import (MERGE_DTYPE, OracleResult, build, criterion_d2, lib_path,  # noqa: F401
                     rhseg)
