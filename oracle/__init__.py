"""CPU FP64 oracle for sign(H_W) b by restarted multishift FOM-LR.

TEST INFRASTRUCTURE ONLY.  This package is the correctness reference: a
plain, slow implementation written from the paper (Bloch et al., "Krylov
subspace methods and the sign function: multishifts and deflation in the
non-Hermitian case", Lattice 2009).  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import it; the library and its
Python binding never do.  It shares no code with the HIP path.

Modules
  dirac      -- H_W = gamma5 D_W(mu): CSR from the definition, free-field FFT form
  rational   -- Kenney-Laub g_s, its partial fractions and first-order poles
  signfun    -- dense sign(A): sorted Schur + Sylvester, Newton (Roberts), eig
  xstar      -- the exact result x* of Algorithm 1 (dense / sparse LU per pole)
  krylov     -- Arnoldi, multishift FOM, restarted FOM-LR (Algorithm 1)
  deflation  -- LR deflation data (dense eig, ARPACK), projector checks
  gradient   -- reference gradients of Re<eta, g(H_W) b>
"""
