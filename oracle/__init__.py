"""CPU oracle for block-floating-point (BFP) multigrid — TEST INFRASTRUCTURE ONLY.

A plain, slow, exact implementation of what the paper's method computes
(Kohl, McCormick, Tamstorf: "Multigrid methods using Block Floating Point
Arithmetic"). Mantissas are arbitrary-precision Python integers held in numpy
object arrays, so no intermediate can overflow; FP64 appears only where the
paper itself works in floating point (the FP64 comparator solver, error norms,
the Chebyshev parameter search).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The HIP library never links, imports or
calls it, and it shares no code with the HIP path; both sides are fed from the
seeded generators in ``workloads``.

Modules
  bfp    — the BFP tuple (Section 2), msb / nu, normalized floor quantization.
  blas   — exact setup/row callbacks (Appendix B), qcomp (Algorithm 1),
           nnqcomp (Algorithm 3), exact dot, normalize, saturate/truncate.
  fd     — finite-difference operators A, R, P after the D=I setup
           (Algorithm "Setup S"), applied on padded grids.
  mg     — Table 1 gamma rules, precision schedules, Chebyshev coefficients,
           IR / V-cycle / FMG in BFP (Appendix C).
  fp64   — FP64 multigrid with the same structure, closed-form discrete
           solutions and error norms.
  cheby  — the empirical eta search for the Chebyshev smoother (Section 5).
"""
