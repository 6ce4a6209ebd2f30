"""FP64 CPU oracle for the DD-DLRA time step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import anything from this package.  The HIP product path never calls it, and
it shares no code with that path (the two only share the seeded input
generators in the separate ``workloads`` module).

Contents
  ddlra        one DD-DLRA step written out from the paper: augmentation
               (Algorithm 4), the projector-splitting integrator for x- and
               y-advection with frozen inflow data (Algorithms 1 and 2, eqs.
               generate_Kboundary and advx_evolK/S/L), truncation (Algorithm
               5), collision/scattering/source (Algorithm 3), the full step
               (Algorithm 6), moments and factored error norms.
  sn_full      the full-tensor S_N scheme (first-order upwind, explicit
               Euler, Lie splitting x / y / collision) that the low-rank
               method approximates; used as an independent reference.
  psi_classic  the single-domain (classic) split projector-splitting
               integrator written in dense-matrix form.

Every function cites the passage it follows.  Places where the paper is
silent, garbled or ambiguous are resolved by readings R1..R22 listed in the
design notes; the ones this code depends on are named where they are used.
"""
