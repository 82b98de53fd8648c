"""Plain FP64 CPU oracle for periodic Parareal with a multi-harmonic coarse correction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its Python
binding) may import, call or link anything in this package; only the test suite,
the smoke check and the CPU-baseline leg of the benchmark use it.  It shares no
code with the GPU path: the only common module is the seeded input generator
``workloads.coax``, which holds none of the method's arithmetic.

Every function cites the passage of the paper (Kulchytska-Ruchka, De Gersem,
Schoeps, "An efficient steady-state analysis of the eddy current problem using a
parallel-in-time algorithm", arXiv:1905.13076) it follows.  Where the paper is
silent the reading taken is named in the docstring.

Parity status per function: every function is pinned by a CPU test against a
closed form, an invariant, a special case or brute force, except the iteration
*histories* of the nonlinear frozen-linearisation coarse rule (``ppc`` on a
nonlinear problem), whose fixed point is pinned but whose per-iteration residuals
are "parity unpinned" by the paper (it defers the nonlinear coarse treatment).  The
alternative nonlinear coarse correction (``nonlinear_coarse_correction``) is pinned
correction by correction: against eq. (4) evaluated row by row with separate coarse
steps, and through its Jacobian against central differences.
"""
