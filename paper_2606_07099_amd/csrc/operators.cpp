#include "operators.h"

#include <algorithm>

#include "sable_pf.h"

namespace sable {

namespace {

// rows and columns of the base kept by an operator, renumbered; -1 = dropped
struct Selection {
  std::vector<int32_t> row, col;
  int32_t rows = 0, cols = 0;
};

void select(const OperatorPattern& B, const Selection& s, bool transpose, OperatorPattern& out) {
  // triplets (new row, new column, base entry) in base order
  std::vector<int32_t> tr, tc, tt;
  for (int32_t r = 0; r < B.rows; ++r) {
    if (s.row[r] < 0) continue;
    for (int32_t t = B.indptr[r]; t < B.indptr[r + 1]; ++t) {
      const int32_t c = s.col[B.indices[t]];
      if (c < 0) continue;
      tr.push_back(s.row[r]);
      tc.push_back(c);
      tt.push_back(t);
    }
  }
  if (transpose) std::swap(tr, tc);
  out.rows = transpose ? s.cols : s.rows;
  out.cols = transpose ? s.rows : s.cols;
  const size_t nnz = tt.size();
  // counting sort by row, stable, so columns stay ascending within a row:
  // the kept rows and columns are monotone renumberings of the base's, and
  // for a transpose the base order visits old rows (new columns) ascending
  out.indptr.assign(out.rows + 1, 0);
  for (size_t k = 0; k < nnz; ++k) out.indptr[tr[k] + 1]++;
  for (int32_t r = 0; r < out.rows; ++r) out.indptr[r + 1] += out.indptr[r];
  std::vector<int32_t> fill(out.indptr.begin(), out.indptr.end() - 1);
  out.indices.assign(nnz, 0);
  out.src.assign(nnz, 0);
  for (size_t k = 0; k < nnz; ++k) {
    const int32_t p = fill[tr[k]]++;
    out.indices[p] = tc[k];
    out.src[p] = tt[k];
  }
  out.pos.assign(B.indices.size(), -1);
  for (size_t p = 0; p < nnz; ++p) out.pos[out.src[p]] = (int32_t)p;
}

}  // namespace

int build_operators(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
                    const int32_t* y_indices, OperatorSet& out, std::string& err) {
  const int32_t n = n_bus;
  std::vector<int32_t> gidx(n, -1), gen;
  int32_t slack = -1;
  for (int32_t i = 0; i < n; ++i) {
    if (bus_type[i] != PF_BUS_PQ) { gidx[i] = (int32_t)gen.size(); gen.push_back(i); }
    if (bus_type[i] == PF_BUS_SLACK) {
      if (slack >= 0) { err = "operators: more than one slack bus"; return PF_EINVAL; }
      slack = i;
    }
  }
  if (slack < 0) { err = "operators: no slack bus"; return PF_EINVAL; }
  const int32_t ng = (int32_t)gen.size();
  const int32_t c_vm = 2 * ng, c_va = 2 * ng + n;

  // ---- the base: rows dP_0..dP_(n-1), dQ_0..dQ_(n-1)
  OperatorPattern& B = out.op[OP_BASE];
  B.rows = 2 * n;
  B.cols = 2 * ng + 2 * n;
  B.indptr.assign(1, 0);
  B.indices.clear();
  out.base.clear();
  std::vector<std::pair<int32_t, int32_t>> row;   // (column bus, Y position)
  for (int32_t half = 0; half < 2; ++half) {
    for (int32_t i = 0; i < n; ++i) {
      row.clear();
      bool diag = false;
      for (int32_t q = y_indptr[i]; q < y_indptr[i + 1]; ++q) {
        const int32_t j = y_indices[q];
        if (j < 0 || j >= n) { err = "operators: Y_bus column out of range"; return PF_EINVAL; }
        if (q > y_indptr[i] && j <= y_indices[q - 1]) { err = "operators: Y_bus row not sorted"; return PF_EINVAL; }
        diag |= j == i;
        row.push_back({j, q});
      }
      if (!diag) {   // dS_i depends on V_i even where Y_ii is structurally zero
        row.push_back({i, -1});
        std::sort(row.begin(), row.end());
      }
      if (gidx[i] >= 0) {
        B.indices.push_back(half * ng + gidx[i]);
        out.base.push_back({BK_SEL, i, i, -1});
      }
      for (const auto& e : row) {
        B.indices.push_back(c_vm + e.first);
        out.base.push_back({half ? BK_DQ_DVM : BK_DP_DVM, i, e.first, e.second});
      }
      for (const auto& e : row) {
        B.indices.push_back(c_va + e.first);
        out.base.push_back({half ? BK_DQ_DVA : BK_DP_DVA, i, e.first, e.second});
      }
      B.indptr.push_back((int32_t)B.indices.size());
    }
  }
  B.src.resize(B.indices.size());
  B.pos.resize(B.indices.size());
  for (size_t t = 0; t < B.indices.size(); ++t) B.src[t] = B.pos[t] = (int32_t)t;

  // ---- F1 rows (dP on B\R, dQ on D) and z1 columns (|V| on D, theta on B\R)
  std::vector<int32_t> ord_p(n, -1), ord_q(n, -1);
  int32_t np = 0, nq = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (bus_type[i] != PF_BUS_SLACK) ord_p[i] = np++;
    if (bus_type[i] == PF_BUS_PQ) ord_q[i] = nq++;
  }
  Selection s1;
  s1.row.assign(B.rows, -1);
  s1.col.assign(B.cols, -1);
  for (int32_t i = 0; i < n; ++i) {
    if (ord_p[i] >= 0) s1.row[i] = ord_p[i];
    if (ord_q[i] >= 0) s1.row[n + i] = np + ord_q[i];
    if (ord_q[i] >= 0) s1.col[c_vm + i] = ord_q[i];
    if (ord_p[i] >= 0) s1.col[c_va + i] = nq + ord_p[i];
  }
  s1.rows = s1.cols = np + nq;
  select(B, s1, false, out.op[OP_J1]);
  select(B, s1, true, out.op[OP_J1T]);

  // ---- J2: rows (dP on R, dQ on B\D), columns (|V|, theta) of every bus
  Selection s2;
  s2.row.assign(B.rows, -1);
  s2.col.assign(B.cols, -1);
  s2.row[slack] = 0;
  for (int32_t k = 0; k < ng; ++k) s2.row[n + gen[k]] = 1 + k;
  for (int32_t c = 0; c < 2 * n; ++c) s2.col[c_vm + c] = c;
  s2.rows = 1 + ng;
  s2.cols = 2 * n;
  select(B, s2, true, out.op[OP_J2T]);

  // ---- J3: rows F1, columns |V| on B\D
  Selection s3;
  s3.row = s1.row;
  s3.col.assign(B.cols, -1);
  for (int32_t k = 0; k < ng; ++k) s3.col[c_vm + gen[k]] = k;
  s3.rows = np + nq;
  s3.cols = ng;
  select(B, s3, true, out.op[OP_J3T]);
  return PF_OK;
}

}  // namespace sable
