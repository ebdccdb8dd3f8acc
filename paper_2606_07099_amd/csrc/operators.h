// The base Jacobian template of one scenario and the operators taken from
// it (host side).  y = (p_g on B\D, q_g on B\D, |V| of every bus, theta of
// every bus) and F = (dP of every bus, dQ of every bus), each block ascending
// by bus (eq. y_and_F_base); J = dF/dy (eq. J_base_block) has constant
// selector entries for the generation columns and the Y_bus pattern in each
// voltage block.  The reduced operators J1, J1^T, J2^T and J3^T (step1_jacobian,
// Jstep2_impl, Jstep3_impl) are its sub-blocks, each with a CSR pattern built
// once and a position map from base entries to its values (the block-aware
// indexing of Sec. III-B).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sable {

enum OperatorId : int { OP_BASE = 0, OP_J1 = 1, OP_J1T = 2, OP_J2T = 3, OP_J3T = 4, OP_COUNT = 5 };

// value kinds of a base entry
enum BaseKind : int { BK_SEL = 0, BK_DP_DVM = 1, BK_DP_DVA = 2, BK_DQ_DVM = 3, BK_DQ_DVA = 4 };

struct BaseEntry {
  int32_t kind;   // BaseKind
  int32_t i, j;   // row bus and column bus (the generator bus for a selector)
  int32_t q;      // Y_bus position of (i, j) in the row-sorted CSR, -1 if absent
};

struct OperatorPattern {
  int32_t rows = 0, cols = 0;
  std::vector<int32_t> indptr, indices;   // CSR, columns sorted within a row
  std::vector<int32_t> src;               // [nnz] base entry of each value
  std::vector<int32_t> pos;               // [nnz of the base] value of each base entry, -1 if unused
};

struct OperatorSet {
  std::vector<BaseEntry> base;            // in the base CSR's value order
  OperatorPattern op[OP_COUNT];
};

// y_indices must be sorted within each row (the template stores it so).
// Returns 0, or PF_EINVAL with err set.
int build_operators(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
                    const int32_t* y_indices, OperatorSet& out, std::string& err);

}  // namespace sable
