"""Oracle: a plain, slow, FP64 CPU statement of what the planning method computes.

This package is TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  The product path (the HIP library
and its Python binding) never imports, calls or links anything here, and this
package imports nothing from the product path: the two share only the seeded
input generator in `synth`, which holds none of the method's arithmetic.

Contents, each following the paper's statement of the method:
  lp       - the weighted-sum LP of App. A (c, A, b, l, u), the preconditioning
             of Sec. 3.C (row normalisation, BOT column scaling beta, the rho
             rule), the primal planning objective F(t) and certified bounds.
  simplex  - a dense bounded-variable primal simplex for min c'x, Ax <= b,
             0 <= x <= u (the exact optimum of every plan).
  vertex   - brute-force vertex enumeration for tiny LPs (pins the simplex).
  admm     - the scaled-form ADMM of Sec. 2.B (Eq. admm with the Schur-complement
             x-step), batched over plans as columns.
  alg1     - Algorithm 1 (overlapping low-dose point sampling), integer exact.
  dose     - dose of a plan at arbitrary voxels and the low-dose band V_j.
"""
