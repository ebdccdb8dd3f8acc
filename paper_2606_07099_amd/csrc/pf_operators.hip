// Value refresh of the Jacobian operators (Algorithm 1 for the entry values,
// the block-aware indexing of Algorithm 2 for their placement), fused: one
// thread per (scenario, value of the operator) reads the base entry that
// feeds the value, evaluates it at the scenario's state and writes it in
// the operator's value order, so the writes are coalesced for transposed
// operators too and no base value buffer is materialised.  A first launch
// forms, once per (scenario, bus), the rectangular voltage e + jf and the
// calculated injection P + jQ that the diagonal entries need.
#include "pf_operators.h"

#include <algorithm>

#include "operators.h"

namespace sable {

__global__ void __launch_bounds__(256) k_operator_state(OpParams p) {
  const size_t o = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= (size_t)p.count * p.n_bus) return;
  const size_t row = o - o % p.n_bus;
  const int i = (int)(o - row);
  double sn, cs;
  sincos(p.va[o], &sn, &cs);
  const double e = p.vm[o] * cs, f = p.vm[o] * sn;
  double ir = 0.0, ii = 0.0;   // I_i = sum_k Y_ik V_k
  for (int k = p.y_rp[i]; k < p.y_rp[i + 1]; ++k) {
    const size_t c = row + p.y_ci[k];
    double sk, ck;
    sincos(p.va[c], &sk, &ck);
    const double ek = p.vm[c] * ck, fk = p.vm[c] * sk;
    ir += p.y_g[k] * ek - p.y_b[k] * fk;
    ii += p.y_g[k] * fk + p.y_b[k] * ek;
  }
  double4 w;
  w.x = e;
  w.y = f;
  w.z = e * ir + f * ii;   // P_i
  w.w = f * ir - e * ii;   // Q_i
  reinterpret_cast<double4*>(p.ef)[o] = w;
}

// F = spec - calc, so every voltage entry is minus the derivative of the
// calculated injection P_i + jQ_i = V_i conj(sum_k Y_ik V_k) (the polar forms
// that Algorithm 1 evaluates, in rectangular products):
//   off the diagonal, with c = V_i V_j cos(theta_ij) = e_i e_j + f_i f_j and
//   s = V_i V_j sin(theta_ij) = f_i e_j - e_i f_j,
//     dP_i/dtheta_j = G s - B c,          dP_i/d|V|_j = (G c + B s) / |V|_j,
//     dQ_i/dtheta_j = -(G c + B s),       dQ_i/d|V|_j = (G s - B c) / |V|_j;
//   on the diagonal, with the row's own P_i and Q_i,
//     dP_i/dtheta_i = -Q_i - B_ii |V_i|^2, dP_i/d|V|_i = P_i / |V|_i + G_ii |V|_i,
//     dQ_i/dtheta_i = P_i - G_ii |V_i|^2,  dQ_i/d|V|_i = Q_i / |V|_i - B_ii |V|_i.
// one value of one scenario
__device__ __forceinline__ double entry_value(const OpParams& p, int kind, int i, int j, double G, double Bv,
                                              size_t b) {
  const double* vm = p.vm + b * p.n_bus;
  const double4* st = reinterpret_cast<const double4*>(p.ef) + b * p.n_bus;
  const double4 si = st[i];
  const double ei = si.x, fi = si.y;
  double dp, dq;   // derivatives of P_i and Q_i
  const bool dva = kind == BK_DP_DVA || kind == BK_DQ_DVA;
  if (i != j) {
    const double4 sj = st[j];
    const double ej = sj.x, fj = sj.y;
    const double c = ei * ej + fi * fj, s = fi * ej - ei * fj;
    if (dva) { dp = G * s - Bv * c; dq = -(G * c + Bv * s); }
    else {
      const double vj = vm[j];
      dp = (G * c + Bv * s) / vj;
      dq = (G * s - Bv * c) / vj;
    }
  } else {
    const double vi = vm[i];
    const double P = si.z, Q = si.w;
    if (dva) { dp = -Q - Bv * vi * vi; dq = P - G * vi * vi; }
    else { dp = P / vi + G * vi; dq = Q / vi - Bv * vi; }
  }
  return -((kind == BK_DP_DVM || kind == BK_DP_DVA) ? dp : dq);
}

// thread = (value of the operator, group of kOpGroup scenarios): the
// pattern-side loads (source map, base entry, Y_bus value) once per group
constexpr int kOpGroup = 8;

__global__ void __launch_bounds__(256) k_operator_values(OpParams p) {
  const size_t o = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t groups = ((size_t)p.count + kOpGroup - 1) / kOpGroup;
  if (o >= groups * p.nnz) return;
  const size_t g = o / p.nnz;
  const int v = (int)(o - g * p.nnz);
  const int t = p.src[v];
  const int4 be = p.base[t];
  const int kind = be.x, i = be.y, j = be.z, q = be.w;
  const double G = (kind != BK_SEL && q >= 0) ? p.y_g[q] : 0.0;
  const double Bv = (kind != BK_SEL && q >= 0) ? p.y_b[q] : 0.0;
  const size_t b1 = min((size_t)p.count, (g + 1) * kOpGroup);
  for (size_t b = g * kOpGroup; b < b1; ++b)
    p.values[b * p.nnz + v] = kind == BK_SEL ? 1.0 : entry_value(p, kind, i, j, G, Bv, b);
}

hipError_t launch_operator_values(const OpParams& p, hipStream_t st) {
  const size_t nst = (size_t)p.count * p.n_bus, total = (size_t)p.count * p.nnz;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_operator_state, dim3((unsigned)((nst + 255) / 256)), dim3(256), 0, st, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t work = ((size_t)p.count + kOpGroup - 1) / kOpGroup * p.nnz;
  hipLaunchKernelGGL(k_operator_values, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, p);
  return hipGetLastError();
}

// Block-diagonal embedding of one scenario's CSR pattern (eq. BDE_global):
// scenario b's block sits at row offset b * rows and column offset b * cols,
// its values at offset b * nnz.  One thread per global row pointer and per
// global column index.
__global__ void __launch_bounds__(256) k_bde_csr(const int* indptr, const int* indices, int rows, int cols,
                                                 int nnz, int count, int64_t* crow, int64_t* col) {
  const size_t o = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t nr = (size_t)count * rows, nc = (size_t)count * nnz;
  if (o <= nr) {
    const size_t b = rows > 0 ? o / rows : 0, r = o - b * rows;
    crow[o] = (o == nr) ? (int64_t)nc : (int64_t)b * nnz + indptr[r];
  }
  if (o < nc) {
    const size_t b = o / nnz, v = o - b * nnz;
    col[o] = (int64_t)b * cols + indices[v];
  }
}

hipError_t launch_bde_csr(const int* indptr, const int* indices, int rows, int cols, int nnz, int count,
                          int64_t* crow, int64_t* col, hipStream_t st) {
  const size_t work = std::max((size_t)count * rows + 1, (size_t)count * nnz);
  hipLaunchKernelGGL(k_bde_csr, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, indptr, indices, rows,
                     cols, nnz, count, crow, col);
  return hipGetLastError();
}

}  // namespace sable

