"""CPU oracle for block-sparse two-site DMRG -- TEST INFRASTRUCTURE ONLY.

This package is the slow, plain, FP64 statement of what the GPU path computes,
written from the paper (Levy, Solomonik, Clark, "Distributed-Memory DMRG via
Sparse and Dense Parallel Tensor Contractions").  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does, and it never imports the product path.

Modules
  blocks    legs, canonical block layout, block tensors, Alg. 2 contraction
  heff      two-site effective Hamiltonian: dense-masked (O1) and block-loop (O2)
  rng       SplitMix64 + Box-Muller Gaussian stream (Davidson restarts)
  eig       Lanczos with full reorthogonalisation; the Davidson routine (Alg. 1)
  truncate  wrapped per-charge SVD split with truncation (Sec. II-C, IV-A)
  env       environment extension and two-site merge (Sec. II-C)
  dmrg      two-site sweeps
  ed        exact diagonalisation (Kronecker / Fock-space constructions)
  grad      reference gradients of E = psi^T H_eff psi
  mpo_dense contraction of an MPO into a dense matrix (to check MPO inputs)

Every function states the passage it follows.  A function without an
independent check says "parity unpinned" in its docstring.
"""
