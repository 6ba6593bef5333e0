"""FP64 CPU oracle for sketched ANLS (DSANLS) -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct restatement of the method of arXiv
2009.02845 in numpy/scipy double precision, used to check the HIP library.
Only the test suite, the smoke entry point and the benchmark's CPU-baseline
leg may import it.  It shares no code with the library (paper_2009_02845_amd)
and never imports it; both sides read their inputs from the seeded generators
in paper_2009_02845_amd/synth.py, which hold none of the method's arithmetic.

Modules:
  philox  -- Philox4x32-10 and the sketch matrices drawn from it (Sec. 3.4)
  dsanls  -- sketch products, prox-CD / PGD updates, objective (Sec. 3.2-3.4)
  mlp     -- FP64 reference of the warm-start network (forward, backward, Adam)

Each function is pinned by tests/test_oracle_*.py against what the paper
and the mathematics fix (known-answer vectors, closed forms, invariants,
brute force, library routines on special cases).  Parity unpinned: the
trajectory of a whole run beyond those pins (the paper prints no values).
"""
