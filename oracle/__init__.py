"""CPU oracle: a plain, slow, FP64 implementation of one time step of the
sharp-interface immersed boundary fractional-step scheme (Vagnoli, Scarpolini,
Verzicco and Viola, "A fast and consistent sharp-interface immersed boundary
method for moving bodies of arbitrary thickness").

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, links or executes it, and
the two share no code: the only common inputs are the seeded arrays built by
the separate ``workloads`` module.

Every function cites the passage of the paper it follows.  Points the paper
leaves open are fixed by explicit readings;
the code states each reading where it is applied.

Modules
  grid        staggered channel grid (Sec. 2, Fig. 1)
  operators   D, G, L_c = DG, viscous L, conservative H (Sec. 2, App. A)
  geometry    closest point on a triangle and the tagging algorithm (Alg. 1),
              boundary/fluid cell classes (Sec. 3.2)
  forcing     two-sided probe and linear reconstruction (Eqs. probe, new_IB)
  linsolve    Thomas and cyclic (Sherman-Morrison) tridiagonal solves
  predictor   explicit RHS and approximate factorisation (Eq. NS_prov)
  poisson     FFT(x) FFT(z) tridiagonal(y) solve of L_c phi = rhs (Eq. elliptic)
  projection  consistent mass correction (Eqs. mod_div .. q_F), projection
              and pressure update (Eqs. projection, update_pressure)
  kinematics  rigid/deforming vertex transforms from host coefficients
  step        one sub-stage and one full time step
  diagnostics no-slip (transpiration) error (Sec. 4.4)
"""
