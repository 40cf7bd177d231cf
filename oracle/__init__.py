"""CPU FP64 oracle for the non-collinear real-time TDDFT step (test infrastructure only).

Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
import this package.  It shares no code with the HIP library and is never on
the product path.  Functions whose result has no independent pin say
"parity unpinned" in their docstring; at present every function is pinned by
a test in tests/test_oracle_pins.py.
"""
