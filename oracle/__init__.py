"""CPU reference (oracle) for adaptive randomized HSS compression.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 numpy/scipy
implementation of what the HIP library computes, written from the paper
"Matrix-free construction of HSS representation using adaptive randomized
sampling" (Gorman, Chavez, Ghysels, Mary, Rouet, Li; arXiv 1810.04125).
It shares no code with the HIP path.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
never does.

Modules
  tree       cluster tree and permutation (Sec. 2.1, the tree figure)
  operators  matrix entries of the synthetic operator families
  hss        Alg. 1-5: local samples, ID, stopping tests, adaptive driver
  matvec     HSS matrix-vector product and reconstruction error
  mlp        4-layer MLP forward / backward / Adam in FP64

Parity unpinned: the safety factor eta on the per-node tolerance and the
readings of the stopping-test details (rho, sqrt(b), the d >= m shortcut)
are pinned only through end-to-end bounds (planted rank, SVD rank
brackets, reconstruction error), not by a value printed in the paper.
"""
