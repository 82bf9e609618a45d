"""CPU oracle: plain, slow, obviously correct BFV multiply+relinearize and bridge.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's
CPU-baseline leg may import, call, link or execute anything in this package.
It shares no code with the HIP library (paper_2204_12201_amd/csrc) and never
imports it; the only thing both sides use is the seeded input module
paper_2204_12201_amd/inputs.py, which holds random draws and parameter sets and
none of the scheme's arithmetic.

Pins: every function is checked in tests/test_oracle_pins.py against
something other than itself (brute force on tiny inputs, exact rational
arithmetic, closed forms and invariants, sympy).  Parity unpinned: the absolute
ciphertext words at full configuration sizes have no external test vector (the
paper prints none); they rest on the pins at small sizes plus the agreement of
two independent implementations.
"""
