"""CPU FP64 oracle for the IgA-SGBEM Galerkin matrix of the 2D Laplace
single-layer operator (Aimi, Calabro, Diligenti, Sampoli, Sangalli, Sestini,
"Efficient assembly based on B-spline tailored quadrature rules for the
IgA-SGBEM").

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s ``cpu_baseline`` leg may import, call, link or execute anything
under ``oracle/``.  It shares no code with the HIP path (no kernels, headers,
helpers or table generators) and imports nothing from it.

Parts:

* ``bspline``, ``curves``: periodic B-spline bases (Cox-de Boor recurrence,
  Section 4.2) and curve evaluation f, f', J (Section 3, eq. J).
* ``circle`` (O1): closed forms on the exact circle (Fourier series of the log
  kernel), used to pin the element-by-element oracle.
* ``ebe`` + ``ebe_oracle.c`` (O2): plain element-by-element assembly, eq.
  elbyelint (Section 5, Remark): tensor Gauss-Legendre on far element pairs,
  regular part Gauss + analytic log part on coincident / adjacent pairs.
* ``nearfield``: reference matrices of the analytic log part, computed in
  50-digit arithmetic from the closed-form base integral of Section 4.2.
* ``wq`` (O3): the weighted-quadrature rules (Alg. 1, Alg. 2, modified moments)
  and the row assembly of eqs. IK1e2 / IK1e2_bis with dense linear algebra.
* ``direct`` (O4): right-hand side of the direct formulation, eq. final_b2
  with the rule of Section 5 (regular weighted outer rule, composite Gauss
  inner rule), F = b1/2 - b2/(2 pi) (eq. seconda_BIE), and the outward flux of
  a harmonic function for the convergence pin.
* ``collocation`` (O5): collocation BEM with the same rules (Conclusions):
  the outer integral replaced by the value at the Greville abscissae.
* ``open_arc``: the singular rule of Section 4.2 on an open interval (the
  paper's own setting of its Table 1 tests).
* ``wq_knots`` (O6): the weighted-quadrature rules and the row assembly on
  non-uniform periodic knots (Section 3): Algorithm 1 per test function,
  Algorithm 2 per source with the full table of singular weights, modified
  moments from the local pieces of the Cox-de Boor recurrence.
* ``wq_open`` (O7): the open arc (Section 2, exterior problem in indirect form;
  Section 3, all N B-splines of the clamped knot vector; Section 4, p + 2 nodes
  in the end elements, minimum-norm end systems; K2 = ln|s - t|), assembled by
  eqs. IK1e2 / IK1e2_bis without mirroring, and the errors E_R, E_M of the
  parabola test (Section 6, Table 2, pinned to the printed values).

Solutions of A alpha = beta (eq. sistlin) in the tests use LAPACK's FP64
solve (numpy) directly; there is no oracle solver of its own.

Every function is FP64 and written for readability, not speed.
"""
