"""Plain, slow CPU FP64 oracle for the ELM-FBPINN block-RRQR + preconditioned-LSQR path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the package entry
module and the CPU-baseline leg of the benchmark may import or call anything in
this package.  The product path (the HIP library and its Python binding) never
does, and shares no code with it: the two meet only in the seeded input arrays
drawn by ``paper_2506_17626_amd.instances``.

Everything is NumPy in float64, written for a reader holding the paper:

* ``assembly`` -- supports, windows, random features, PDE operators and the
  weighted rows of the global system (Section 2.1, eq. elm_solution,
  eq. fcn_depth_h, eq. ELMFBPINN_ls, eq. DomainDecomp; Section 4.2, eq. dd and
  eq. used_window_function_nd).
* ``rrqr`` -- the sigma-RRQR filter of Algorithm 1 as classical column-pivoted
  Householder QR with exact norm recomputation, stopping relative to the
  leading diagonal of R.
* ``lsqr`` -- the right-preconditioned operator of Proposition 3.1 (Q form and
  R form) and LSQR (Paige and Saunders 1982) as used by Algorithm 2.
* ``solve`` -- back-substitution a = S^{-1} y with zeros at dropped columns
  (Algorithm 2, output step), evaluation of the ansatz and the normalised L1
  error (Section 4.2, performance evaluation).
* ``forms`` -- the mixed-precision refinement form and the MLP warm-start
  network (forward, backward, Adam) used to check the GPU forms.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms, invariants, library routines on special cases and brute force;
functions without such a pin are flagged "parity unpinned" in their docstring.
"""
