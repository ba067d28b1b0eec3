"""CPU FP64 oracle for the plane-wave block-LOBPCG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library and
its Python binding) may import, call, link or execute anything in this package.
Only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

Contents (each function cites the passage of Bottin, Leroux, Knyazev, Zerah,
"Large scale ab initio calculations based on three levels of parallelization",
Comput. Mater. Sci. 2007, that it follows):

  pw.py       plane-wave sphere, kinetic diagonal, DFT of the local potential,
              Kleinman-Bylander projectors, the dense Galerkin Hamiltonian
              (sec. 2.1: the expansion of the wave-function over plane waves
              and the projected eigenproblem), the overlap operator O of the
              generalized form and its Cholesky reduction to one Hermitian
              matrix, and the electron density.
  jacobi.c    cyclic complex-Hermitian Jacobi diagonalisation (plain C, FP64,
              single-threaded, no BLAS) -- the oracle's eigensolver.
  jacobi.py   ctypes loader for jacobi.c (built by __graft_entry__.build()).
  matfree.py  matrix-free H.X through numpy FFTs, the block LOBPCG of
              sec. 3.2 (Algorithm 1, with O = I or the overlap operator) run
              block by block with the constraint to previous blocks, the final
              Rayleigh-Ritz over all bands, and residual certificates.  Paper-scale reference and CPU baseline.

Parity pins: every function here is checked in tests/test_oracle_*.py against
closed forms, lattice counts, library special cases or brute force, never
against itself.  Functions without such a pin say "parity unpinned".
"""
