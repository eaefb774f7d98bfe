"""Plain FP64 CPU oracle for near-circulant splitting (NCS).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library (no
kernels, headers, tables, constants or helpers); the only thing both sides use
is the seeded input generator in ``ncs_inputs``, which holds none of the
method's arithmetic.

Everything here is written from the paper (Ryu, Ko, Won, "Splitting with
Near-Circulant Linear Systems: Applications to Total Variation CT and PET"):

* ``projector``  -- the discrete Radon transform as an explicit sparse matrix
  (Section 4.1.1 says only "discretization of the Radon transform"; the
  Joseph ray-driven model is the reading used on both sides).
* ``operators``  -- the finite-difference matrices of Section 2 and the
  circulant multipliers of Section 4.1.1 (eq. circ_R, eq. circ_D).
* ``prox``       -- the proximal maps: Moreau identity (Section 2), box
  projection and quadratic prox (Section 4.1), the Poisson map S
  (Section 4.2), and the per-pixel l2-ball projection for isotropic TV.
* ``objective``  -- the CT and PET objectives, KKT residuals and the
  D-seminorm of Section 3.3.
* ``solvers``    -- NCS (eq. NCS and its CT/PET forms in Section 4), PDHG
  (eq. PDHG), ADMM in the reduced form (eq. ADMM) and in the classic form of
  the appendix.
* ``problems``   -- assembling seeded synthetic problems.
* ``fanbeam``    -- the fan-beam projector and the probe estimate of
  eq. (H-fan) (Section 4.1.1).
* ``conebeam``   -- the cone-beam projector on volumes, 3D differences, the 3D
  multiplier and the NCS iteration on volumes (Section 4.1.1).

Parity status of each function is stated in its docstring; every function is
pinned by a ``-m "not gpu"`` test against closed forms, special cases,
invariants or brute force, except the definitional choices listed as
"parity unpinned" in ``problems``.
"""
