// Device-side value refresh of the base Jacobian template and of the
// operators taken from it (one scenario's pattern, values for a batch).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "sable_pf.h"

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

// the batch-global CSR of the block-diagonal embedding of one scenario's
// pattern (indptr[rows + 1], indices[nnz], device) for `count` scenarios:
// crow[count * rows + 1], col[count * nnz] (device, int64)
hipError_t launch_bde_csr(const int* indptr, const int* indices, int rows, int cols, int nnz, int count,
                          int64_t* crow, int64_t* col, hipStream_t st);

// launch parameters of operator `which` of a template, except the per-bus
// state buffer `ef`; validates the arguments and sets the pf_last_error
// message on failure (PF_OK or a PF_E* code); device: the template's
int operator_params(pf_template* t, int which, int count, const double* vm, const double* va, double* values,
                    const char* name, OpParams& p, int& device);
// message returned by pf_last_error on this thread
void set_error(const std::string& msg);

}  // namespace sable
