"""libovderiv for MI355X: two-sided Lanczos sgn(H(mu)) b, its derivative by the
block-matrix method and generalised deflation (arXiv:1611.00195), as HIP
kernels behind a C ABI.  Import ``paper_1611_00195_amd.ovderiv`` for the
Python binding; importing this package itself needs no GPU."""
