"""FP64 CPU oracle for the compressed-VIE solve — TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct NumPy implementation of what
the GPU path computes: the discretised volume integral equation Z I = v0
(paper §3, eq. 3.6), its dense product, dense LU solve, the block-diagonal
preconditioner (§4, eqs. 4.1-4.2), left-preconditioned restarted GMRES (§6,
the GMRES setting), the near/far recursive grouping (§5.1, §5.3, §5.4) and the
checks that certify low-rank factors (§5.2, eq. 5.3; §6.2 accuracy metrics).

It shares no code with the HIP library and never imports it.  Only the tests,
the smoke entry point and the benchmark's CPU-baseline leg may import it; the
product path must never route through it.

Each module header lists the tests that pin its functions against the paper or the
mathematics (closed forms, invariants, brute force, special cases).
"""
from . import discretise, greens, grouping, solvers, compressed  # noqa: F401
