"""Plain FP64 CPU oracle for the forced relativistic lattice Boltzmann (RLBM) step.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or links
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, tables or
constants with the HIP library; the only thing both sides consume is the
seeded input generators in ``workloads/``, which hold none of the method's
arithmetic.

The oracle follows the paper (M. Watson, "Two Dimensional Turbulence in a
Massless Fluid with a Relativistic Lattice Boltzmann Model", arXiv:2101.06187)
step by step, in the paper's order and notation, vectorised over lattice sites
with NumPy and written for a reader to check by eye, not for speed:

  (b) stream the populations by linear interpolation   -- ``rlbm.stream``
  (c) moments T^{mu nu}                                 -- ``rlbm.moments``
      Landau frame eigenproblem for eps, u              -- ``rlbm.landau``
  (d) truncated Juettner equilibrium                    -- ``rlbm.equilibrium``
  (e) Anderson-Witting collision                        -- ``rlbm.collide``
      projected stirring-force term                     -- ``rlbm.force_source``

Modules:
  stencil      momentum stencils (spherical 26-direction set; 8-direction circle)
  philox       Philox4x32-10 counter-based generator (Salmon et al., SC'11)
  forcing      stirring-force modes and the configuration-space force field
  rlbm         one time step and its stages
  diagnostics  fields, conserved sums, energy spectrum and enstrophy

Every function states which passage of the paper it follows and, where the
paper is silent or garbled, which reading it takes.  Pins that tie the oracle
to something other than itself live in ``tests/test_oracle_*.py``.
"""

from . import stencil, philox, forcing, rlbm, diagnostics  # noqa: F401
