"""FP64 CPU oracle for randomized CP decomposition (Erichson, Manohar,
Brunton, Kutz: "Randomized CP Tensor Decomposition").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path
and is written from the paper alone:

  philox     Philox4x32-10 counter-based generator and the Gaussian test
             matrix Omega_n built from it (Section 3.1, Algorithm 1's test-matrix draw).
  rcp        the randomized compression (Algorithm 1), CP-ALS on the core
             (Algorithm 2), back-projection (eq. qbs), the fit of
             Section 3.3 and deterministic CP-ALS (the same solver with
             Q_n = I).
  evaluate   relative reconstruction error (Section 4) and factor
             congruence for comparing two Kruskal tensors.

Everything is float64 NumPy / SciPy.  Each function cites the passage it
follows.  Parity status of every function is listed in its docstring;
all are pinned by the oracle self-tests.
"""
