"""CPU float64 oracle for the quantics-MPS Fresnel propagation path.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_2510_23089_amd``) never imports, calls or links anything here, and
nothing here imports the product package; the two share only the seeded input
generators in ``synth``.

Every function is a plain, slow, direct transcription of the definition it
cites (numpy / scipy in float64 / complex128; LAPACK SVD and numpy FFT serve as
library steps).  The pins that tie each function to the paper or to
mathematics, independently of the code itself, live in ``tests/test_oracle_*``.

Modules
-------
quantics  bit-interleaved index map (Sec. 3, "quantics representation")
ttsvd     sequential SVD construction of an MPS (Sec. 4, App. A) and the keep rule
fresnel   dense FFT Fresnel propagation (Sec. 6.1, paraxial transfer function)
mpo       dense operators -> MPO by interleaved SVD (Sec. 6.1, MPO construction
          figure), bit-reversed DFT (Sec. 5), axis embedding
zipup     MPO x MPS zip-up contraction, truncation sweep, rounding, decompression
refine    two-site variational fitting sweep (one FP32 refinement pass reading)
grad      torch-CPU complex128 twin of zipup/sweep/decompress for autograd

Parity status: every function above is pinned by at least one test in
``tests/test_oracle_*.py``; see the docstrings for which.  The truncating
zip-up is pinned in closed form for operators of bond 1 (single-site
unitaries on a left-canonical input: the right-to-left sequential truncated
SVD of the exact result, i.e. the TT-SVD of the site-reversed vector), and
with operator bonds above 1 by brute force on 8-site chains (the definition
evaluated densely, without the carry recursion).
"""
