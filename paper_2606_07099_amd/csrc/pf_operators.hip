// Value refresh of the Jacobian operators (Algorithm 1 for the entry values,
// the block-aware indexing of Algorithm 2 for their placement), fused: one
// thread per (scenario, value of the operator) reads the base entry that
// feeds the value, evaluates it at the scenario's state and writes it in
// the operator's value order, so the writes are coalesced for transposed
// operators too and no base value buffer is materialised.
#include "pf_operators.h"
#include "operators.h"

namespace sable {

namespace {

__device__ __forceinline__ void voltage(const double* vm, const double* va, int k, double& e, double& f,
                                        double& v) {
  double s, c;
  sincos(va[k], &s, &c);
  v = vm[k];
  e = v * c;
  f = v * s;
}

}  // namespace

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
__global__ void __launch_bounds__(256) k_operator_values(OpParams p) {
  const size_t o = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= (size_t)p.count * p.nnz) return;
  const size_t b = o / p.nnz;
  const int t = p.src[o - b * p.nnz];
  const int4 be = p.base[t];
  const int kind = be.x, i = be.y, j = be.z, q = be.w;
  double val = 1.0;   // selector
  if (kind != BK_SEL) {
    const double* vm = p.vm + b * p.n_bus;
    const double* va = p.va + b * p.n_bus;
    const double G = q >= 0 ? p.y_g[q] : 0.0, Bv = q >= 0 ? p.y_b[q] : 0.0;
    double ei, fi, vi;
    voltage(vm, va, i, ei, fi, vi);
    double dp, dq;   // derivatives of P_i and Q_i
    const bool dva = kind == BK_DP_DVA || kind == BK_DQ_DVA;
    if (i != j) {
      double ej, fj, vj;
      voltage(vm, va, j, ej, fj, vj);
      const double c = ei * ej + fi * fj, s = fi * ej - ei * fj;
      if (dva) { dp = G * s - Bv * c; dq = -(G * c + Bv * s); }
      else { dp = (G * c + Bv * s) / vj; dq = (G * s - Bv * c) / vj; }
    } else {
      double ir = 0.0, ii = 0.0;
      for (int k = p.y_rp[i]; k < p.y_rp[i + 1]; ++k) {
        double ek, fk, vk;
        voltage(vm, va, p.y_ci[k], ek, fk, vk);
        ir += p.y_g[k] * ek - p.y_b[k] * fk;
        ii += p.y_g[k] * fk + p.y_b[k] * ek;
      }
      const double P = ei * ir + fi * ii, Q = fi * ir - ei * ii;
      if (dva) { dp = -Q - Bv * vi * vi; dq = P - G * vi * vi; }
      else { dp = P / vi + G * vi; dq = Q / vi - Bv * vi; }
    }
    val = -((kind == BK_DP_DVM || kind == BK_DP_DVA) ? dp : dq);
  }
  p.values[o] = val;
}

hipError_t launch_operator_values(const OpParams& p, hipStream_t st) {
  const size_t total = (size_t)p.count * p.nnz;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_operator_values, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace sable
