"""CPU FP64 oracle for the derivative of sgn(H(mu)) b -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow reference that the GPU library is checked
against.  It is imported only by the tests, by ``__graft_entry__.smoke()`` and
by the ``cpu_baseline`` leg of ``bench.py``; the library itself never imports,
links or calls it, and the two share no code (only the seeded input generators
in ``synth`` feed both).

Modules
  dirac      Wilson-Dirac kernel H(mu) = gamma5 Dw(mu), its adjoint and its
             derivatives in mu and along a link tangent (Sec. 1, eq. 1).
  matfun     matrix sign by spectral form / Schur / Newton, and the Frechet
             derivative through the block matrix of eq. 6 (Sec. 2).
  tsl        two-sided Lanczos Krylov-Ritz approximation of f(A)x, and its
             application to the block matrix B of eq. 6-7 (Sec. 2).
  deflation  standard (eq. 8) and generalised (eq. 9-11) deflation, eigenpairs
             and eigenvector derivatives (Sec. 3).
  vjp        gradient of the bilinear <x|sgn(H)|b> with respect to mu and to
             every link (the fermionic force the paper motivates in Sec. 1).
  freefield  exact sgn(H)b for unit links in momentum space (any lattice size).
  estimator  the error estimate eps_A of Sec. 4.

Parity status: every function here is pinned by tests in ``tests/`` against
something other than itself (dense linear algebra, closed forms, identities,
finite differences); see each module's docstring.
"""
