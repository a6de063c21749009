"""FP64 CPU oracle for the matrix-free spectral/hp elemental operators.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code with the HIP library (no tables, helpers or constants);
the two meet only through the seeded input generators, which hold none of
the method's arithmetic.

What it computes is the plain definition, written out with explicit dense
matrices and no sum-factorisation:

* 1-D quadrature (Gauss-Lobatto-Legendre, Gauss-Radau-Jacobi) - ``quadrature``
* modified C0 Jacobi bases of hex, prism and tet - ``basis``
* element maps, Jacobians and metric terms - ``geometry``
* BwdTrans u = B u^, IProductWRTBase u^ = B^T W f, PhysDeriv,
  IProductWRTDerivBase, and the Helmholtz operator H = L + lambda M
  (paper section 2.1, eqs. (5)-(9); section 2.2, eqs. (14)-(23)) - ``operators``
* structured-hex C0 assembly and Jacobi-preconditioned CG - ``assembly``
* a tiny sum-factorised brute force written from eqs. (16), (17), (20), (21),
  (22), used only to cross-check the explicit matrices - ``sumfac``

Equation numbers follow the order of the displayed equations in the paper:
(1) Helmholtz PDE, (5) matrix form, (6) H = L + lambda M, (7) L and M,
(8) basis matrix, (9) physical derivative, (13) collapsed coordinates,
(14)-(15) backward transform, (16)/(17) its sum-factorised hex/tet forms,
(18) tet mode map, (19) inner product, (20)/(21) its sum-factorised hex/tet
forms, (22) standard derivative, (23) eta-to-xi chain rule, (24) throughput.
"""
