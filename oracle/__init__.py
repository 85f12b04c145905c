"""CPU oracle for the sum-over-Cliffords hot path (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product package never imports it.
"""
from .oracle import *  # noqa: F401,F403
