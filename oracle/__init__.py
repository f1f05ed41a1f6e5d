"""Plain FP64 CPU oracle for the domain-decomposed Newmark field update.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; the two
see the same seeded input arrays (from the `workloads` package) and nothing
else.

What it computes (the paper's Sec. IV-A states that the decomposed fields
equal the monolithic ones to near machine precision, so the oracle is the
monolithic solve):
  * its own canonical edge numbering and PEC classification (fem.py);
  * lowest-order Whitney edge-element mass and curl-curl matrices, written
    out from the definition of the 1-form basis (Sec. II-B-1) (fem.py);
  * the global, undecomposed Newmark-beta recurrence (Sec. II-B-2) for the
    edge-only wave equation, each step solved with a sparse direct
    factorisation (SuperLU through scipy, a library primitive) (newmark.py);
  * the discrete Gauss law, the discrete energy and the reverse-mode adjoint
    of the recurrence (newmark.py);
  * the particle steps around the solve (Sec. II-A): point location, the
    exact current mapping of straight paths onto the edges, Whitney
    interpolation of E and B at points, Faraday's per-tetrahedron update of
    B and the Adams-Bashforth push (pic.py);
  * the mixed E/B system on edges and faces (Whitney 2-forms, the discrete
    curl, the face mass) advanced by the trapezoid rule as one monolithic
    block solve (mixed.py).

Parity status: every function here is pinned by a test that does not
re-use its own formula (see tests/test_oracle_*.py).
"""
