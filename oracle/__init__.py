"""FP64 CPU oracle for Chebyshev-filtered subspace iteration on the
spectral finite-element Kohn-Sham Hamiltonian (DFT-FE 1.0, arXiv 2203.07820).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path:
it has its own quadrature tables, its own mesh numbering helpers, its own
assembly and its own solver.  Both sides only read the same seeded inputs
from ``workloads``.

Modules
-------
``fe``      spectral-element tables, operator assembly (Section 2.3,
            discrete Hamiltonian and Loewdin transform), cell-wise H.X
            (Section 4.3, cell-level products and assembly).
``chfsi``   Lanczos upper bound, scaled Chebyshev filter (Section 3.1),
            Cholesky-Gram-Schmidt and Rayleigh-Ritz (Algorithm 2), the pass
            loop.
``mlp``     the warm-start network: forward, backward, subspace loss, Adam.

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms (free-electron spectra,
constant shifts, the explicit Chebyshev polynomial), dense LAPACK
eigendecompositions, invariants and finite differences.  The continuum
accuracy of the Gaussian-atom systems has no closed form (parity unpinned
beyond self-convergence in p).
"""
