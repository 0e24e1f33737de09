"""Plain, slow, float64 CPU oracle for the LeanVec search path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the package's smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the GPU library; the only
common inputs are the seeded arrays from ``synth``.

Modules (each function cites the passage of the paper it follows):

* ``exact``    -- maximum-inner-product ground truth (Section 2, notation).
* ``lvq``      -- per-vector scale/bias scalar quantiser (LVQ; cited in
                  Section 2, defined here by the reading in the module text).
* ``fit``      -- second moments, LeanVec-ID (Section 2.1), the LeanVec-OOD
                  loss, its trace form and gradients (Section 2.2-2.3),
                  the Frank-Wolfe block coordinate descent (Algorithm 1) and
                  the eigenvector search (Section 2.4, Algorithm 2).
* ``search``   -- greedy graph traversal on primary vectors and re-ranking
                  with secondary vectors (Section 2 "Search", Appendix D).
* ``projloss`` -- sampled-pair refinement loss and its gradients, built from
                  the LeanVec-OOD objective (Problem leanvec_orthonormal).

Parity status: every function is pinned by tests under ``tests/`` against
closed forms, brute force or invariants; see the module headers.
"""
