"""FP64 CPU oracle for randomized CP-ALS (CPRAND / CPRAND-MIX).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import or call anything here; the GPU
library never does, and this package imports nothing from it.

Plain, slow and written for checking by eye against Battaglino, Ballard and
Kolda, "A Practical Randomized CP Tensor Decomposition": every function cites
the section, equation or algorithm it follows.  numpy/scipy supply the
library steps (SVD-based least squares, FFT, SVD, matrix products).

Modules:
  philox    Philox4x64-10 and the method's random draws (samples, signs, fit set)
  tensor    unfolding, Kronecker / Khatri-Rao products, CP reconstruction, TTM
  cprand    SKR, fiber sampling, sampled LS, mixing, fit, stop rules, the ALS loops
  leverage  leverage scores, coherence, Khatri-Rao leverage and its marginals
  score     factor-match score
  proposal  integer proposals and importance-weighted sampling
  mlp       the learned proposal network (forward, backward, Adam) and its features

Parity status: every function is pinned by a CPU test against something
other than itself (a closed form, an identity, a brute-force enumeration, a
library routine or a number printed in the paper), except where a module
header says "parity unpinned".
"""
