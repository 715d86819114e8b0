"""FP64 CPU oracle for randomized Tucker with Kronecker sketches.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the benchmark's CPU-baseline leg, never by the product library or its
binding.  It shares no code with the HIP path.

Parity pins: every public function is checked by ``tests/test_oracle_*.py``
against closed forms, brute force, paper-printed values and invariants.
The only unpinned choices are listed in ``oracle.tucker``'s header (the
assignment of subrank factors to modes in the sequentially truncated
algorithm).
"""
from . import tucker, lowp, adjoint  # noqa: F401
