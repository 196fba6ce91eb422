"""FP64 CPU oracle for the HODLR-preconditioned GMRES path.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct NumPy/SciPy code
written from the paper (Aminfar, Ambikasaran & Darve, "A Fast Block Low-Rank
Dense Solver with Applications to Finite-Element Matrices", arXiv:1403.5337)
and, where the paper only cites a method, from that method's published
definition.  It is used by ``tests/``, by the smoke check and by the CPU
baseline leg of the benchmark; the product path never imports it.  It shares
no code with the GPU library: only the seeded input generators in ``gen``
feed both.

Modules
  tree      index-range tree of the HODLR structure (Sec. 4.1)
  ordering  recursive coordinate bisection of the separator dofs
  aca       partial-pivoting adaptive cross approximation (Sec. 5.1)
  bdlr      boundary-distance pseudo-skeleton (Sec. 5.3, eq. Ahat)
  hodlr     HODLR assembly, Woodbury factorization and solve (Sec. 4.2-4.3)
  gmres     flexible right-preconditioned GMRES (Sec. 3)
  cg        preconditioned conjugate gradients for the symmetric fronts (Sec. 3)
  dense     dense LU reference solve
  mlp       the skeleton scorer's network, loss, gradient and Adam (float64)
  features  the scorer's per-vertex features and training labels

Parity status of each function is stated in its module docstring.
"""
