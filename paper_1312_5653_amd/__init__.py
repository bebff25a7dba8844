"""sfdp: range-space Schur solve of Poisson-constrained distributed control with
the complex factorization S = conj(Z) M^-1 Z, Z = K + i beta^(-1/2) M, each
factor solved by FETI-DP on one MI355X (HIP kernels behind a C ABI).

The native library is loaded lazily by ``paper_1312_5653_amd.sfdp``; importing
this package does not load it.
"""
