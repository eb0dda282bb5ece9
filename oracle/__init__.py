"""Plain, slow FP64 CPU oracle for the screened-interaction hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, link or
call anything in this folder; only the tests, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code, header, table or
constant with the GPU library.

Paper: D. Foerster, P. Koval, D. Sanchez-Portal, "An O(N^3) implementation of
Hedin's GW approximation for molecules" (arXiv:1101.2065).  Every function in
gw_oracle.py names the section and equation it follows.

Pinning (tests/test_oracle_pins.py): every function is checked against facts
the paper or the mathematics fixes (closed forms, sum rules, moments, symmetry,
brute force on tiny inputs, a grid number the paper prints).  Nothing here is
"parity unpinned".
"""
from .gw_oracle import *  # noqa: F401,F403
