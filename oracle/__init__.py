"""Independent CPU oracle for the Leuvenshtein hot path -- TEST INFRASTRUCTURE.

Plain, slow, obviously correct reference used to check the HIP library.  It
shares no code with ``paper_2508_14568_amd`` (they meet only in the seeded
input generators of ``workloads``).  Only ``tests/``, the package smoke check
and the benchmark's CPU-baseline leg may import it; the product path never
does.

Modules:
  plaintext    -- Wagner-Fischer, the difference-encoded DP, the lookup tables.
  tfhe         -- schoolbook TFHE in Z/2^64 (C core in tfhe_ref.c).
  leuvenshtein -- Algorithms 3/4 and the Section 5 preprocessing, encrypted.

Parity status: every function is pinned by a test against the paper's printed
values, closed forms or brute force, except the exact ciphertext bits, which
no published value fixes (they are guarded by decryption, invariants and the
agreement of two independent implementations).
"""
