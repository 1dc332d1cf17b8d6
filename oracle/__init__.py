"""Plain FP64 CPU oracle for the two-site effective Hamiltonian and the local LCC solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its Python
binding) imports, links or runs this package; only the tests, the `__graft_entry__.smoke()`
check and the CPU-baseline leg of the benchmark do.  It shares no code with the GPU path:
the only common module is `workloads`, which generates the seeded inputs.

Modules
  fock        O1: the Hamiltonian built directly from second quantisation in the Fock
              space of one (N, 2Sz) sector, the MPS contracted into explicit basis vectors,
              and H_eff = P^T H P (the derivative graph with the local tensor removed,
              Implementation section, local-derivative figure).  Small systems only.
  mpo         the oracle's own matrix product operator (MPO equation): a plain prefix
              automaton over the Hamiltonian's operator strings, Jordan-Wigner signs
              explicit.
  blocksparse O2: environments and the two-site H_eff x by an explicit block sum
              (transition-element figure), any system size the CPU can hold.
  solve       the local linear problem (first-order equation of the RS hierarchy, local
              Hylleraas functional) solved densely or by plain FP64 conjugate gradients,
              Lanczos for shifts.

Parity notes: every function states which passage of the paper it follows.  Functions
whose result has no independent pin say so ("parity unpinned") in their docstring.
"""
