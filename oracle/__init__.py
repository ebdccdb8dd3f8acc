"""CPU FP64 correctness oracle for batched Newton-Raphson AC power flow.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
GPU library never imports, links or calls this package, and this package
never imports the GPU library: the two share no code.  The only shared module
is ``gen`` (seeded synthetic inputs, no power-flow arithmetic).

Contents (plain, slow, dense; every function cites the passage it follows):

* :mod:`oracle.ybus`      -- pi-model bus admittance matrix (dense complex).
* :mod:`oracle.newton`    -- Step-1 Newton completion per scenario, dense
  Jacobian from the complex-matrix derivative forms, LAPACK ``gesv``.
* :mod:`oracle.adjoint`   -- implicit-differentiation gradients by a dense
  transposed solve, the training loss, and central finite differences.
* :mod:`oracle.completion` -- Step-2 explicit recovery of the generation
  outputs and the gradients of the whole two-step completion (vbar2 through
  a dense J2, then the Step-1 transposed solve).
* :mod:`oracle.operators` -- the base Jacobian template dF/dy with its
  selector blocks and the operators J1, J1^T, J2^T, J3^T as dense sub-blocks.

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
invariants, finite differences, the paper's printed Jacobian entries
(Algorithm 1) and brute-force root finding.
"""
