"""CPU FP64 reference ("oracle") for the Stokes-preconditioned BEFE step.

TEST INFRASTRUCTURE ONLY. Nothing in the library imports, calls or links this
package; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark do. It is a plain, slow, direct transcription of the discrete
problem the library solves, written from the paper's description:

* Phi_dt(u) = (I - dt L)^{-1} (u + dt N(u)), the Backwards-Euler /
  Forwards-Euler step (Sec. 2, eq. befe), with the boundary conditions,
  incompressibility and pressure carried by the implicit solve (Sec. 2,
  after eq. befe; Sec. 3.2 for the influence-matrix requirement that the
  result be divergence free to machine accuracy);
* Fourier x Chebyshev x Fourier discretisation with pseudospectral products
  (Sec. 3.2), dealiased by the 3/2 rule in x and z;
* the Newton update U <- U - u with G_U u = G(U) (Sec. 2, eqs. linear and
  biglin), solved by unrestarted GMRES (Sec. 2, eq. Kspace);
* the exact linearisation N -> N_U with homogeneous boundary conditions
  (Sec. 2, after eq. factor2) and its adjoint.

Modules:
  grid      -- mode numbers and wavenumbers of the canonical layout
  cheb      -- Chebyshev points, synthesis/analysis, derivative, Gram matrix
  fourier   -- padded inverse / truncated forward FFTs in x and z
  stokes    -- the per-mode coupled Chebyshev-tau Stokes system, solved densely
  befe      -- N(u), Phi, residual, norms, JVP, VJP
  krylov    -- GMRES (modified Gram-Schmidt, Givens) and Newton
  pack      -- canonical complex layout <-> packed real vector
  gint      -- the multi-step time-integration operator (BEFE or SBDF2 steps)
  advect    -- the implicit operator with the laminar advection added
  symmetry  -- the shift-reflect projector of plane Couette flow

Every function is pinned by a CPU test against something other than itself
(closed forms, analytic Stokes eigenvalues, brute-force products, library
routines, exact identities of the method); see each module's header.
"""
