"""CPU oracle for the batched candidate evaluation of Plessen's GPU heuristic
search for multi-tour biomass logistics (arXiv 1909.10286).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It is a plain, slow, obviously correct reference,
written from the paper: exact Python integers for every decision (supplies in
kg, distances in metres, times in seconds) and float64 for the reported cost
in km.  It shares no code with the HIP library; the only thing both take is
the seeded input generator ``paper_1909_10286_amd.inputs``, which holds none
of the method's arithmetic.

Modules:
  philox   - counter-based Philox generator (Salmon et al., SC'11).
  model    - supplies, shuttle drives, tour geometry, times, cost (sec. 2.1-2.3,
             eqs. (1)-(5)); the HU and SU min-max rebalancing (sec. 2.5, Alg. 2);
             feasibility (eq. (2)); candidate key and gate (sec. 2.5).
  init     - initial solution of Algorithm 1 and its feasibility (sec. 2.5).
  moves    - Alg. 1's remove-and-reinsert moves drawn from Philox (sec. 2.5).
  search   - Algorithm 1, GPU version, with the eq. (6) exploration rule.
  surrogate- float64 set-encoder network used to check the learned screen.

Parity status: every function is pinned by tests under tests/ (closed forms,
brute force on tiny inputs, invariants, library routines); the paper publishes
no instance or worked example, so parity with the paper's own numbers is
unpinned.
"""
