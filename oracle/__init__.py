"""Plain CPU reference ("oracle") for the Benchmark-Streaming operations.

TEST INFRASTRUCTURE ONLY.  Nothing in the library path imports, links or
calls this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP library; the two meet
only through the seeded inputs of ``bsgen``.

Everything here is binary64 numpy (plus ``math.fsum``), written to be read
against the paper (Chalmers & Warburton, "Portable high-order finite element
kernels I: Streaming Operations"):

  ops    -- the seven streaming operations of Table 1 (BS1-BS7)
  mesh   -- the structured hex mesh, its scatter map Z (eq. scatter_def),
            the CSR form of the gather operator Z^T, node degrees, weights
  model  -- the launch-latency + bandwidth model, its least-squares fit and
            the Fischer-Brown point (eqs. time_model, perf_model,
            Fischer-Brown)
  cg     -- conjugate gradients (Algorithm 1) on a 7-point operator, and
            mixed-precision iterative refinement around it
  batch  -- one step of the batched workload (the seven operations and one
            CG iteration) on one box-mesh instance
  elem   -- the element operators of Section 2 (GLL Lagrange basis, mass
            and stiffness blocks, their assembly Z^T A_L Z, lumped mass)
"""

from . import batch, cg, elem, mesh, model, ops  # noqa: F401
