"""Plain, slow FP64 CPU oracle for entropy-variable hybridized DG.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The GPU library never calls it and shares no code with it: the
reference-element tables, geometry, physics, Jacobians and linear algebra here
are written independently (Vandermonde bases, numpy Gauss rules, cross-product
face normals, complex-step derivatives, LAPACK solves), so an error in either
side shows up as a parity failure.

Modules:

* ``refelem``  -- nodes, quadrature rules and Lagrange bases per element type
* ``geometry`` -- affine / multilinear maps, Jacobians, face normals
* ``physics``  -- entropy variables, inviscid and viscous fluxes, trace fluxes
* ``hdg``      -- element residual, complex-step Jacobian, static condensation,
                  trace operator, brute-force global solve, back-solve
* ``krylov``   -- GMRES(m) with optional right preconditioner, block-Jacobi
* ``mlp``      -- a small NumPy multilayer perceptron with hand-written backward

Every function cites the part of the paper it follows.  Parity pins (tests
under ``tests/test_oracle_*.py``) tie each part to something other than itself.
"""
