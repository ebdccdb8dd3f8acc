// Device-side value refresh of the base Jacobian template and of the
// operators taken from it (one scenario's pattern, values for a batch).
#pragma once

#include <hip/hip_runtime.h>

namespace sable {

struct OpParams {
  const int4* base;      // [nnz_base] {kind, i, j, q} (BaseKind, bus pair, Y_bus position)
  const int* src;        // [nnz] base entry of each value of the operator
  const int *y_rp, *y_ci;
  const double *y_g, *y_b;
  const double *vm, *va; // [count][n_bus] state of each scenario
  double* ef;            // [count][n_bus] (e, f, P, Q): e + jf = V, P + jQ = V conj(I), formed first
  double* values;        // [count][nnz]: the value array of the batch-global (block-diagonal) CSR
  int nnz, n_bus, count;
};

// two launches on st: the per-bus state, then the values
hipError_t launch_operator_values(const OpParams& p, hipStream_t st);

}  // namespace sable
