"""FP64 CPU oracle for the 4-D spectral-convolution FNO block.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check in
__graft_entry__.py and by the cpu_baseline leg of bench.py, never by the
product package.  See oracle/fno_oracle.c for the definitions and the
paper passages they follow.
"""
from .oracle import *  # noqa: F401,F403
