"""CPU oracle (test infrastructure only).

Plain FP64 reference implementations written from the paper.  Only the
tests, ``__graft_entry__.smoke`` and the benchmark's CPU-baseline leg may
import this package; the product path never does.
"""
