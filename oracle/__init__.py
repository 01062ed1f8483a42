"""CPU FP64 oracle for the overlapping solution-transfer DD method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It is a plain, slow, obviously-correct
implementation written from the paper; it shares no code with the HIP path
(the only shared module is the seeded input generator ``problems``).

Modules
-------
fd       finite-difference model problem (Section 2.1, model problem of eq. basic)
dd       solution-transfer blocks (eq. defS), equivalent loads (eq. equilib1),
         equilibrium system (eq. modelS), interface solve, volume recovery
gmres    plain unrestarted GMRES with modified Gram-Schmidt (Section 5)
hodlr    weak-admissibility hierarchical low-rank reference (Section 2.4)
adjoint  discrete adjoint gradient w.r.t. the cellwise coefficient

Parity status: every function is pinned by CPU tests (tests/test_oracle_*.py)
against values the paper prints, closed forms, invariants or brute force.
"""
