"""Plain FP64 CPU oracle for the per-level AMR time step of the axion-string field.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library never
links, imports or calls it, and it shares no code, tables or helpers with the HIP
path; both take their initial states from the separate ``synth`` package.

What it computes, and from where (paper: arXiv 2404.02950, "sledgehamr"):

* ``scalars``  -- level spacing/time step (section II, eqs. for Delta x_l and
  eq. dtscaling), stage times of classic RK4 (integrator type 4, appendix E table
  "Integrator settings"), the EOM coefficients (minimal example, eq. EOM2).
* ``level``    -- the 7-point Laplacian (appendix A, order 1), the right-hand side of
  eqs. EOM1/EOM2 and one classic RK4 step on a periodic dense lattice.
* ``energy``   -- the lattice energy (kinetic + forward-difference gradient +
  potential), the quantity appendix B uses to measure convergence.
* ``tagging``  -- the problem-specific tagging hook (section "Problem-specific cell
  tagging") instantiated as plaquette winding of the phase of psi1 + i psi2.
* ``amr``      -- Berger-Oliger subcycling (section II.A and Fig. 2), coarse-to-fine
  ghost interpolation in space and time (section II.A; linear conservative
  interpolation, appendix E table "AMR parameters", type 1) and level
  synchronisation by averaging fine onto coarse.
* ``layout``   -- checks of a box layout: blocking-factor alignment, maximum box size,
  cover of the buffered tags and proper nesting (sections II and II.C).

Arrays are indexed ``[z, y, x]``; a state is ``(4, nz, ny, nx)`` = (psi1, psi2, Pi1, Pi2).
Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
