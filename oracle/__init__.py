"""Plain FP64 CPU oracle of the cell-centred Lagrangian ADER-WENO finite volume
scheme with time-accurate local time stepping (Boscheri, Dumbser, Zanotti,
arXiv:1408.3719).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or calls
this package: only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code with the HIP library; the two meet only at the
seeded inputs built by the ``workloads`` package.

Pins (tests/test_oracle_*.py): closed-form quadrature and basis tables, exact
reproduction of degree-M polynomials by the reconstruction, exact predictor
solutions (constant state, entropy wave, rigid translation), node-solver
translation, closed space-time volumes (GCL), free stream on a deforming
mesh with local time steps, conservation at every cycle, deadlock freedom,
LTS with one level against a separate GTS driver, the Sod problem against an
exact Riemann solver and the design order on the smooth vortex; the
reverse-mode step against the NumPy step, central differences of it and the
conservation identity of its adjoint.

Parity unpinned (definitions the paper leaves to its references; they are
checked only by the invariants above and by agreement with the GPU path):
the stencil shapes, the equispaced space-time nodal set, the number of
Picard sweeps and the quadrature orders.

Layout
  tables.py    universal reference-element tables (quadrature, bases, time matrices)
  topology.py  edges, rings, face neighbours, the 7 WENO stencils, scheduling stencils
  euler.py     Euler fluxes and the ideal-gas equation of state (eulerTerms, eqn.eos)
  scheme.py    reconstruction, predictor, node solver, space-time patch fluxes,
               update, local time step, the LTS cycle driver and a separate GTS driver
  adjoint.py   one global step on a fixed mesh with dt held fixed, in PyTorch CPU
               FP64 ops, differentiated by torch.autograd (reverse-mode oracle)
"""
