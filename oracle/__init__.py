"""ORACLE -- test infrastructure only.

Plain, slow, obviously correct CPU references for what the GPU path
computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU path
(``paper_2506_15183_amd``); the seeded input generators in
``paper_2506_15183_amd.scenes`` are the one thing both sides use.
"""
