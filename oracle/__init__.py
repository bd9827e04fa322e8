"""Correctness oracle for the Eulerian-Eulerian six-scheme lattice Boltzmann
step (Piredda & Asinari, arXiv:2409.10399).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or run it.  The product
path (``paper_2409_10399_amd``) never imports it and shares no code, table or
constant with it.

Everything here is plain NumPy in FP64: one time step at a time, in the order
the paper describes it, with the boundary rules of its Sec. 3.5 and the
readings stated beside each line for what the paper leaves open.

Functions and what pins them (tests under ``tests/test_oracle_*.py``):

* ``equilibria.feq_I / feq_S / feq_L`` -- moment identities (Eqs. (37), (42),
  (50), (72), (80)) on D1Q3/D2Q9/D3Q19 and the printed D1Q3 closed forms of
  Appendix A (typed from the paper in ``tests/test_oracle_equilibria.py``).
* ``scheme.Oracle.step`` -- uniform rest state is a fixed point; the uniform
  drift-flux state of Eq. (124) is a fixed point (buoyancy, drag, Clift-Grace-
  Weber factor); uniform slip relaxation follows its closed-form recurrence
  and conserves mixture momentum; periodic budgets (sum of the sources is zero,
  per-phase eps and alpha conserved); dashpot + lag recurrence of Eqs. (128),
  (131), (133); single-phase Taylor-Green decay against the closed form;
  Gaussian volume-fraction pulse against the analytic advection-diffusion
  solution with the diffusivity of Eq. (88); the mixture sound speed implied by
  Eqs. (19), (20), (32); D2Q9 with y-uniform fields projecting exactly onto
  D1Q3; mirror symmetry.
* Boundary rules of Sec. 3.5 in several dimensions (walls, corners) --
  parity unpinned: the paper has no multi-dimensional boundary data; they are
  checked only for the 1D steady relations and for symmetry.
* ``fd.FD`` -- a finite-difference method-of-lines solver of the same
  two-fluid artificially compressible system (Sec. 3.4 in several dimensions,
  classical Runge-Kutta in time), pinned by closed forms in
  ``tests/test_oracle_fd.py`` (budgets, drift-flux fixed point, slip
  relaxation, Taylor-Green decay, mixture sound speed, advected Gaussian,
  weighted shear momentum); the LBM oracle approaches it at second order under
  the diffusive refinement of Sec. 2.1.2 (16^2 / 32^2 / 64^2 boxes, all four
  fields), which ties the coupled PDE content of ``scheme.Oracle.step`` --
  sources, stress, volume-fraction force, drag, buoyancy together -- to an
  independent discretisation.
* ``mapping`` -- the similarity numbers printed for TEST #4 and the TEST #1
  outlet relations (``tests/golden/test4_mapping.json``,
  ``tests/golden/test1_outlet.json``).
"""
from .lattice import CS2, Lattice, d1q3, d2q9, d3q19, by_name  # noqa: F401
from .scheme import Oracle, Params, spalding_B  # noqa: F401
