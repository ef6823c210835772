"""CPU oracle for SFA regular-expression matching — TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, independently written implementation of what
the matcher computes.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product package never does,
and the two share no code (only the seeded input generators in
``workloads``, which hold no matching arithmetic).

What the matcher computes has a plain definition: the state reached by the
minimal complete DFA of the regex after reading every input byte from its
start state, and whether that state is accepting (sequential computation of a
DFA, Algorithm 2 of Section 2; membership w in L(A) by the definitions of
computation and accepted language in Section 2.2).  States are reported in the
canonical numbering (breadth-first from the start state, bytes 0..255 in
ascending order, numbered in order of discovery), so that two independent
constructions can be compared state by state.

Modules
-------
``regex``     byte-regex parser and a set-of-positions matcher built straight
              from the language definitions (no automata).
``automata``  Thompson NFA, subset construction (Algorithm 1, Section 2.3),
              Moore minimisation, canonical numbering, byte classes.
``sfa``       D-SFA correspondence construction (Algorithm 4, Section 5.1 with
              the deterministic simplification), the reverse composition of
              Section 2.1, parallel SFA computation (Algorithm 5, Section 5.2)
              and speculative DFA simulation (Algorithm 3, Section 3).
``nsfa``      the SFA built from an NFA: position automaton (Glushkov), the
              NFA run from I, Algorithm 4 over correspondences Q -> P(Q),
              composition of correspondences and Algorithm 5 with
              S_fin = union of f_fin(q) over q in I.
``scan``      Algorithm 2 in plain C (``seqscan.c``) and Algorithm 5 on host
              threads in plain C (``cpu_sfa.c``) for large inputs.
``build``     compiles ``seqscan.c`` and ``cpu_sfa.c`` with gcc.

Every function that is not pinned against something other than itself says
"parity unpinned" in its docstring; the pins live in ``tests/test_oracle_*.py``.
"""
from .regex import parse, ParseError, matches  # noqa: F401
from .automata import compile_regex, Dfa  # noqa: F401
from .sfa import build_dsfa, Dsfa, OverCap  # noqa: F401
