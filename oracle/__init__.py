"""CPU oracle for the recursive sparse LU (spaLU) of Zhu & Lai (2024).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 definition
of what the factorization computes: nested dissection with segment
structure (Section 3, Algorithm 1, specialised to regular grids), leaf
elimination, per-level hybrid-sampled interpolative decompositions and
Schur sparsification, segment LU, separator elimination and merging
(Section 4, Algorithm 2), the solve x = V~ W~ b, and iterative refinement.
Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the GPU library never does, and the two share no
code.

Functions whose result is not pinned by a check other than itself say
"parity unpinned" in their docstring.
"""
