// Device kernels of the batched Newton power flow for CDNA4 (gfx950).
//
// One workgroup owns one scenario for the whole Newton solve (no host round
// trip per iteration): complex Y_bus SpMV + mismatch, convergence test,
// Jacobian value evaluation fused into a row-oriented 2x2-block LU
// refactorisation on the fixed symbolic pattern (forward solve fused), the
// level-scheduled backward solve, FP64-residual refinement in the mixed
// precision mode, and the state update.  Small grids keep every per-scenario
// array in LDS; large grids keep them in the per-scenario HBM workspace and
// stage only the row being factorised in LDS.
#include "pf_kernels.h"

#include <hip/hip_runtime.h>

namespace sable {

// ----------------------------------------------------------------------------
// small helpers

struct B4d { double v[4]; };

template <typename T>
struct Blk { T a, b, c, d; };  // row-major 2x2 block [[a, b], [c, d]]

template <typename T>
__device__ __forceinline__ Blk<T> ld_blk(const T* p) { return {p[0], p[1], p[2], p[3]}; }
template <typename T>
__device__ __forceinline__ void st_blk(T* p, const Blk<T>& x) { p[0] = x.a; p[1] = x.b; p[2] = x.c; p[3] = x.d; }

template <typename T>
__device__ __forceinline__ Blk<T> mul(const Blk<T>& x, const Blk<T>& y) {
  return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}

// Jacobian entries of J1 = dF1/dz1 for the bus pair (i, m): rows (dP_i, dQ_i),
// columns (theta_m, |V|_m).  Written in rectangular coordinates V = e + jf,
// I = Y V: for i != m the products |V_i||V_m| cos(theta_im) = e_i e_m + f_i f_m
// and |V_i||V_m| sin(theta_im) = f_i e_m - e_i f_m replace the trigonometric
// terms; the values equal the closed forms of Algorithm 1.
__device__ __forceinline__ B4d jac_entries(int i, int m, double G, double B, const double* e,
                                           const double* f, const double* vm, const double* ire,
                                           const double* iim) {
  B4d r;
  if (i == m) {
    double ei = e[i], fi = f[i], v = vm[i];
    double P = ei * ire[i] + fi * iim[i];
    double Q = fi * ire[i] - ei * iim[i];
    double v2 = v * v;
    r.v[0] = Q + B * v2;
    r.v[1] = -P / v - G * v;
    r.v[2] = -P + G * v2;
    r.v[3] = -Q / v + B * v;
  } else {
    double cc = e[i] * e[m] + f[i] * f[m];
    double ss = f[i] * e[m] - e[i] * f[m];
    double gs_bc = G * ss - B * cc;
    double gc_bs = G * cc + B * ss;
    double vmm = vm[m];
    r.v[0] = -gs_bc;
    r.v[1] = -gc_bs / vmm;
    r.v[2] = gc_bs;
    r.v[3] = -gs_bc / vmm;
  }
  return r;
}

// The 2x2 block of the padded block system at LU position p of block row a.
// PV buses keep a dummy |V| unknown and a dummy dQ row: identity on the
// diagonal, zero coupling; fill-in positions start at zero.
template <typename T>
__device__ __forceinline__ Blk<T> fill_block(const DevSym& s, int a, int p, const double* e,
                                             const double* f, const double* vm, const double* ire,
                                             const double* iim) {
  const int src = s.lu_src[p];
  const int j = s.ci[p];
  const bool dg = (j == a);
  if (src < 0 && !dg) return {T(0), T(0), T(0), T(0)};
  const int i = s.blk_bus[a], m = s.blk_bus[j];
  const double G = src < 0 ? 0.0 : s.y_g[src];
  const double Bv = src < 0 ? 0.0 : s.y_b[src];
  B4d x = jac_entries(i, m, G, Bv, e, f, vm, ire, iim);
  const bool pv_i = s.bus_type[i] == 1, pv_m = s.bus_type[m] == 1;
  if (pv_i) { x.v[2] = 0.0; x.v[3] = 0.0; }
  if (pv_m) { x.v[1] = 0.0; x.v[3] = 0.0; }
  if (dg && pv_i) x.v[3] = 1.0;
  return {T(x.v[0]), T(x.v[1]), T(x.v[2]), T(x.v[3])};
}

__device__ __forceinline__ int pick_group(int nrows, int nt, int gmin) {
  int g = 64;
  while (g > gmin && (nt / g) < nrows) g >>= 1;
  return g;
}

template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ----------------------------------------------------------------------------
// per-scenario context: pointers into LDS or into the HBM workspace

template <typename T>
struct Ctx {
  double *e, *f, *vm, *va, *ire, *iim, *ps, *qs, *dvr, *dvi, *aux;  // [n_bus]
  double *F, *dx, *rr;                                        // [2 nb]
  T *y;                                                       // [2 nb]
  T *lu, *dinv;                                               // [4 nnzb], [4 nb]
  T *wsp;                                                     // row workspaces (HBM mode)
  double* red;                                                // [nwaves]
  int* flags;                                                 // [nwaves + 4]
};

template <typename T>
__device__ void bind_state(Ctx<T>& c, double* d, T* t, const StateLayout& L) {
  c.e = d + L.o_e; c.f = d + L.o_f; c.vm = d + L.o_vm; c.va = d + L.o_va;
  c.ire = d + L.o_ire; c.iim = d + L.o_iim; c.ps = d + L.o_ps; c.qs = d + L.o_qs;
  c.dvr = d + L.o_dvr; c.dvi = d + L.o_dvi; c.aux = d + L.o_aux;
  c.F = d + L.o_F; c.dx = d + L.o_dx; c.rr = d + L.o_rr;
  c.y = t + L.o_y; c.lu = t + L.o_lu; c.dinv = t + L.o_dinv;
}

// max over the workgroup of v, OR of bad; every thread gets the result
__device__ double block_max(double v, int bad, int* bad_out, double* red, int* flags, int tid, int nt) {
  for (int o = 32; o > 0; o >>= 1) {
    v = fmax(v, __shfl_xor(v, o));
    bad |= __shfl_xor(bad, o);
  }
  const int w = tid >> 6;
  if ((tid & 63) == 0) { red[w] = v; flags[w] = bad; }
  __syncthreads();
  double m = 0.0;
  int b = 0;
  for (int k = 0; k < (nt >> 6); ++k) { m = fmax(m, red[k]); b |= flags[k]; }
  __syncthreads();
  *bad_out = b;
  return m;
}

// ----------------------------------------------------------------------------
// phases (each ends with a workgroup barrier)

// I = Y V, S = V conj(I), F1 = spec - calc on the block rows; returns ||F1||_inf.
template <typename T>
__device__ double phase_mismatch(const DevSym& s, Ctx<T>& c, int tid, int nt, int* bad_out) {
  double mx = 0.0;
  int bad = 0;
  for (int i = tid; i < s.n_bus; i += nt) {
    double ir = 0.0, ii = 0.0;
    for (int q = s.y_rp[i]; q < s.y_rp[i + 1]; ++q) {
      const int j = s.y_ci[q];
      const double g = s.y_g[q], b = s.y_b[q];
      const double ej = c.e[j], fj = c.f[j];
      ir += g * ej - b * fj;
      ii += g * fj + b * ej;
    }
    c.ire[i] = ir;
    c.iim[i] = ii;
    const int a = s.bus_blk[i];
    if (a >= 0) {
      const double ei = c.e[i], fi = c.f[i];
      const double P = ei * ir + fi * ii;
      const double Q = fi * ir - ei * ii;
      const double F0 = c.ps[i] - P;
      const double F1 = s.bus_type[i] == 0 ? c.qs[i] - Q : 0.0;
      c.F[2 * a] = F0;
      c.F[2 * a + 1] = F1;
      bad |= !(isfinite(F0) && isfinite(F1));
      mx = fmax(mx, fmax(fabs(F0), fabs(F1)));
    }
  }
  __syncthreads();
  return block_max(mx, bad, bad_out, c.red, c.flags, tid, nt);
}

// Row-oriented block LU of one row (Doolittle by rows): fill the row's J1
// values, eliminate it against the finished rows k in L(a,:) in increasing
// order (L_ak = A_ak U_kk^-1; A_aj -= L_ak U_kj for j in U(k,>k)), apply the
// same L_ak to the right-hand side (forward solve), and invert the pivot
// block.  The G lanes of one group share the row; all of them belong to one
// wavefront, whose LDS operations complete in program order, so a value one
// lane writes in step k is seen by every lane in step k+1.
template <typename T, bool LDS>
__device__ void factor_row(const DevSym& s, Ctx<T>& c, int a, int lane, int G, T* W, bool fill,
                           bool fwd) {
  const int rs = s.rp[a], re = s.rp[a + 1], dg = s.diag[a];
  const int len = re - rs;
  if (fill) {
    for (int q = lane; q < len; q += G)
      st_blk(W + 4 * q, fill_block<T>(s, a, rs + q, c.e, c.f, c.vm, c.ire, c.iim));
  } else if (!LDS) {
    for (int q = lane; q < len; q += G) st_blk(W + 4 * q, ld_blk(c.lu + 4 * (rs + q)));
  }
  T y0 = T(0), y1 = T(0);
  if (fwd) { y0 = c.y[2 * a]; y1 = c.y[2 * a + 1]; }
  for (int p = rs; p < dg; ++p) {
    const int k = s.ci[p];
    const int q = p - rs;
    const Blk<T> A = ld_blk(W + 4 * q);
    const Blk<T> L = mul(A, ld_blk(c.dinv + 4 * k));
    if (fwd) {
      const T yk0 = c.y[2 * k], yk1 = c.y[2 * k + 1];
      y0 -= L.a * yk0 + L.b * yk1;
      y1 -= L.c * yk0 + L.d * yk1;
    }
    const int ks = s.diag[k] + 1;
    const int n = s.rp[k + 1] - ks;
    const int ts = s.upd_start[p];
    for (int t = lane; t < n; t += G) {
      const Blk<T> U = ld_blk(c.lu + 4 * (ks + t));
      T* w = W + 4 * s.upd_tgt[ts + t];
      Blk<T> x = ld_blk(w);
      const Blk<T> LU = mul(L, U);
      x.a -= LU.a; x.b -= LU.b; x.c -= LU.c; x.d -= LU.d;
      st_blk(w, x);
    }
    if (lane == 0) st_blk(W + 4 * q, L);
  }
  if (lane == 0) {
    const Blk<T> D = ld_blk(W + 4 * (dg - rs));
    const T det = D.a * D.d - D.b * D.c;
    const T inv = T(1) / det;
    const Blk<T> Di = {D.d * inv, -D.b * inv, -D.c * inv, D.a * inv};
    // pivots of the block: a, then the Schur complement d - c b / a
    const T p1 = D.a, p2 = det / D.a;
    const T eps = sizeof(T) == 8 ? T(1e-14) : T(1e-7);
    const bool zero = !(fabs(p1) > eps * (fabs(D.a) + fabs(D.b))) ||
                      !(fabs(p2) > eps * (fabs(D.c) + fabs(D.d))) || !isfinite(inv);
    if (zero) c.flags[kZeroPivotFlag] = 1;
    st_blk(c.dinv + 4 * a, Di);
    if (fwd) { c.y[2 * a] = y0; c.y[2 * a + 1] = y1; }
  }
  if (!LDS) {
    for (int q = lane; q < len; q += G) st_blk(c.lu + 4 * (rs + q), ld_blk(W + 4 * q));
  }
}

template <typename T, bool LDS>
__device__ void phase_factor(const DevSym& s, Ctx<T>& c, int tid, int nt, int gmin, int wstride,
                             bool fill, bool fwd) {
  for (int lev = 0; lev < s.nlev_l; ++lev) {
    const int r0 = s.lev_l_ptr[lev], r1 = s.lev_l_ptr[lev + 1];
    const int G = pick_group(r1 - r0, nt, gmin);
    const int gid = tid / G, lane = tid % G, ng = nt / G;
    for (int ri = r0 + gid; ri < r1; ri += ng) {
      const int a = s.lev_l_rows[ri];
      T* W = LDS ? c.lu + 4 * s.rp[a] : c.wsp + (size_t)gid * wstride;
      factor_row<T, LDS>(s, c, a, lane, G, W, fill, fwd);
    }
    __syncthreads();
  }
}

// L y = y (unit block-lower, in place) by L-levels
template <typename T>
__device__ void phase_fsolve(const DevSym& s, Ctx<T>& c, int tid, int nt, int gmin) {
  for (int lev = 0; lev < s.nlev_l; ++lev) {
    const int r0 = s.lev_l_ptr[lev], r1 = s.lev_l_ptr[lev + 1];
    const int G = pick_group(r1 - r0, nt, gmin);
    const int gid = tid / G, lane = tid % G, ng = nt / G;
    for (int ri = r0 + gid; ri < r1; ri += ng) {
      const int a = s.lev_l_rows[ri];
      T s0 = T(0), s1 = T(0);
      for (int p = s.rp[a] + lane; p < s.diag[a]; p += G) {
        const Blk<T> L = ld_blk(c.lu + 4 * p);
        const int k = s.ci[p];
        const T y0 = c.y[2 * k], y1 = c.y[2 * k + 1];
        s0 += L.a * y0 + L.b * y1;
        s1 += L.c * y0 + L.d * y1;
      }
      s0 = group_sum(s0, G);
      s1 = group_sum(s1, G);
      if (lane == 0) { c.y[2 * a] -= s0; c.y[2 * a + 1] -= s1; }
    }
    __syncthreads();
  }
}

// U x = y (block-upper with full diagonal blocks, in place) by U-levels
template <typename T>
__device__ void phase_bsolve(const DevSym& s, Ctx<T>& c, int tid, int nt, int gmin) {
  for (int lev = 0; lev < s.nlev_u; ++lev) {
    const int r0 = s.lev_u_ptr[lev], r1 = s.lev_u_ptr[lev + 1];
    const int G = pick_group(r1 - r0, nt, gmin);
    const int gid = tid / G, lane = tid % G, ng = nt / G;
    for (int ri = r0 + gid; ri < r1; ri += ng) {
      const int a = s.lev_u_rows[ri];
      T s0 = T(0), s1 = T(0);
      for (int p = s.diag[a] + 1 + lane; p < s.rp[a + 1]; p += G) {
        const Blk<T> U = ld_blk(c.lu + 4 * p);
        const int j = s.ci[p];
        const T x0 = c.y[2 * j], x1 = c.y[2 * j + 1];
        s0 += U.a * x0 + U.b * x1;
        s1 += U.c * x0 + U.d * x1;
      }
      s0 = group_sum(s0, G);
      s1 = group_sum(s1, G);
      if (lane == 0) {
        const Blk<T> D = ld_blk(c.dinv + 4 * a);
        const T t0 = c.y[2 * a] - s0, t1 = c.y[2 * a + 1] - s1;
        c.y[2 * a] = D.a * t0 + D.b * t1;
        c.y[2 * a + 1] = D.c * t0 + D.d * t1;
      }
    }
    __syncthreads();
  }
}

// U^T w = g (in place in y) by L-levels: w_a = U_aa^-T (g_a - sum_k U_ka^T w_k)
template <typename T>
__device__ void phase_ut_solve(const DevSym& s, Ctx<T>& c, int tid, int nt, int gmin) {
  for (int lev = 0; lev < s.nlev_l; ++lev) {
    const int r0 = s.lev_l_ptr[lev], r1 = s.lev_l_ptr[lev + 1];
    const int G = pick_group(r1 - r0, nt, gmin);
    const int gid = tid / G, lane = tid % G, ng = nt / G;
    for (int ri = r0 + gid; ri < r1; ri += ng) {
      const int a = s.lev_l_rows[ri];
      T s0 = T(0), s1 = T(0);
      for (int p = s.rp[a] + lane; p < s.diag[a]; p += G) {
        const Blk<T> U = ld_blk(c.lu + 4 * s.mirror[p]);  // U_ka, k = ci[p]
        const int k = s.ci[p];
        const T w0 = c.y[2 * k], w1 = c.y[2 * k + 1];
        s0 += U.a * w0 + U.c * w1;
        s1 += U.b * w0 + U.d * w1;
      }
      s0 = group_sum(s0, G);
      s1 = group_sum(s1, G);
      if (lane == 0) {
        const Blk<T> D = ld_blk(c.dinv + 4 * a);
        const T t0 = c.y[2 * a] - s0, t1 = c.y[2 * a + 1] - s1;
        c.y[2 * a] = D.a * t0 + D.c * t1;
        c.y[2 * a + 1] = D.b * t0 + D.d * t1;
      }
    }
    __syncthreads();
  }
}

// L^T l = w (in place in y) by U-levels: l_a = w_a - sum_j L_ja^T l_j
template <typename T>
__device__ void phase_lt_solve(const DevSym& s, Ctx<T>& c, int tid, int nt, int gmin) {
  for (int lev = 0; lev < s.nlev_u; ++lev) {
    const int r0 = s.lev_u_ptr[lev], r1 = s.lev_u_ptr[lev + 1];
    const int G = pick_group(r1 - r0, nt, gmin);
    const int gid = tid / G, lane = tid % G, ng = nt / G;
    for (int ri = r0 + gid; ri < r1; ri += ng) {
      const int a = s.lev_u_rows[ri];
      T s0 = T(0), s1 = T(0);
      for (int p = s.diag[a] + 1 + lane; p < s.rp[a + 1]; p += G) {
        const Blk<T> L = ld_blk(c.lu + 4 * s.mirror[p]);  // L_ja, j = ci[p]
        const int j = s.ci[p];
        const T l0 = c.y[2 * j], l1 = c.y[2 * j + 1];
        s0 += L.a * l0 + L.c * l1;
        s1 += L.b * l0 + L.d * l1;
      }
      s0 = group_sum(s0, G);
      s1 = group_sum(s1, G);
      if (lane == 0) { c.y[2 * a] -= s0; c.y[2 * a + 1] -= s1; }
    }
    __syncthreads();
  }
}

// dV = V (d|V|/|V| + j dtheta) for the correction dx (slack: 0)
template <typename T>
__device__ void phase_dv(const DevSym& s, Ctx<T>& c, int tid, int nt) {
  for (int i = tid; i < s.n_bus; i += nt) {
    const int a = s.bus_blk[i];
    double dvr = 0.0, dvi = 0.0;
    if (a >= 0) {
      const double dth = c.dx[2 * a];
      const double rho = s.bus_type[i] == 0 ? c.dx[2 * a + 1] / c.vm[i] : 0.0;
      dvr = c.e[i] * rho - c.f[i] * dth;
      dvi = c.f[i] * rho + c.e[i] * dth;
    }
    c.dvr[i] = dvr;
    c.dvi[i] = dvi;
  }
  __syncthreads();
}

// r = -F1 - J1 dx in FP64 without forming J1: J1 dx = -(dS restricted to the
// F1 rows), dS = dV conj(I) + V conj(Y dV).  Result cast into y.
template <typename T>
__device__ void phase_residual(const DevSym& s, Ctx<T>& c, int tid, int nt) {
  for (int i = tid; i < s.n_bus; i += nt) {
    const int a = s.bus_blk[i];
    if (a < 0) continue;
    double dir = 0.0, dii = 0.0;
    for (int q = s.y_rp[i]; q < s.y_rp[i + 1]; ++q) {
      const int j = s.y_ci[q];
      const double g = s.y_g[q], b = s.y_b[q];
      dir += g * c.dvr[j] - b * c.dvi[j];
      dii += g * c.dvi[j] + b * c.dvr[j];
    }
    const double e = c.e[i], f = c.f[i], ir = c.ire[i], ii = c.iim[i];
    const double dvr = c.dvr[i], dvi = c.dvi[i];
    const double dSr = dvr * ir + dvi * ii + e * dir + f * dii;
    const double dSi = dvi * ir - dvr * ii + f * dir - e * dii;
    const double r0 = -c.F[2 * a] + dSr;
    const double r1 = s.bus_type[i] == 0 ? -c.F[2 * a + 1] + dSi : 0.0;
    c.rr[2 * a] = r0;
    c.rr[2 * a + 1] = r1;
    c.y[2 * a] = T(r0);
    c.y[2 * a + 1] = T(r1);
  }
  __syncthreads();
}

// adjoint residual r = g - J1^T lam in FP64 without forming J1 (transposed
// directional derivative of S = V conj(Y V)): with nu = lam_P + j lam_Q and
// c_m = conj(nu_m I_m) + sum_i Y_im nu_i conj(V_i),
//   (J1^T lam)_theta_m = Im(V_m c_m),  (J1^T lam)_|V|m = -Re(V_m c_m) / |V_m|.
// Also stores Re(V_m c_m) / |V_m| = -(J3^T lam)_m for every bus in aux.
// g == nullptr: only aux is produced.
template <typename T>
__device__ void phase_adj_residual(const DevSym& s, Ctx<T>& c, int tid, int nt,
                                   const double* lam, const double* g, bool to_y) {
  for (int i = tid; i < s.n_bus; i += nt) {   // w_i = nu_i conj(V_i) -> (dvr, dvi)
    const int a = s.bus_blk[i];
    double nr = 0.0, ni = 0.0;
    if (a >= 0) { nr = lam[2 * a]; ni = s.bus_type[i] == 0 ? lam[2 * a + 1] : 0.0; }
    c.dvr[i] = nr * c.e[i] + ni * c.f[i];
    c.dvi[i] = ni * c.e[i] - nr * c.f[i];
  }
  __syncthreads();
  for (int m = tid; m < s.n_bus; m += nt) {
    double tr = 0.0, ti = 0.0;
    for (int q = s.y_rp[m]; q < s.y_rp[m + 1]; ++q) {
      const int i = s.y_ci[q];
      const int qt = s.y_tr[q];              // position of Y_im
      const double yg = s.y_g[qt], yb = s.y_b[qt];
      tr += yg * c.dvr[i] - yb * c.dvi[i];
      ti += yg * c.dvi[i] + yb * c.dvr[i];
    }
    const int a = s.bus_blk[m];
    double nr = 0.0, ni = 0.0;
    if (a >= 0) { nr = lam[2 * a]; ni = s.bus_type[m] == 0 ? lam[2 * a + 1] : 0.0; }
    const double ir = c.ire[m], ii = c.iim[m];
    const double cr = (nr * ir - ni * ii) + tr;      // Re c_m
    const double ci = -(nr * ii + ni * ir) + ti;     // Im c_m
    const double e = c.e[m], f = c.f[m];
    const double vcr = e * cr - f * ci;               // Re(V_m c_m)
    const double vci = e * ci + f * cr;               // Im(V_m c_m)
    c.aux[m] = vcr / c.vm[m];
    if (a >= 0 && g) {
      const double r0 = g[2 * a] - vci;
      const double r1 = s.bus_type[m] == 0 ? g[2 * a + 1] + vcr / c.vm[m] : 0.0;
      c.rr[2 * a] = r0;
      c.rr[2 * a + 1] = r1;
      if (to_y) { c.y[2 * a] = T(r0); c.y[2 * a + 1] = T(r1); }
    }
  }
  __syncthreads();
}

template <typename T>
__device__ void phase_set_state(const DevSym& s, Ctx<T>& c, int tid, int nt) {
  for (int i = tid; i < s.n_bus; i += nt) {
    double sn, cs;
    sincos(c.va[i], &sn, &cs);
    c.e[i] = c.vm[i] * cs;
    c.f[i] = c.vm[i] * sn;
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// the Newton kernel: one workgroup = one scenario

template <typename T, bool LDS>
__global__ void __launch_bounds__(1024) k_newton(KParams kp) {
  extern __shared__ __align__(16) unsigned char smem[];
  const DevSym& s = kp.s;
  const int b = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const StateLayout& L = kp.lay;

  double* gd = kp.ws_d + (size_t)b * L.sd;
  T* gt = reinterpret_cast<T*>(kp.ws_t) + (size_t)b * L.st;
  int* gi = kp.ws_i + (size_t)b * 4;

  Ctx<T> c;
  c.red = reinterpret_cast<double*>(smem);
  c.flags = reinterpret_cast<int*>(smem + kRedBytes);
  unsigned char* dyn = smem + kScratchBytes;
  if (LDS) {
    bind_state<T>(c, reinterpret_cast<double*>(dyn),
                  reinterpret_cast<T*>(dyn + 8 * (size_t)L.sd), L);
    c.wsp = nullptr;
  } else {
    bind_state<T>(c, gd, gt, L);
    c.wsp = reinterpret_cast<T*>(dyn);
  }
  int* zflag = c.flags + kZeroPivotFlag;
  if (tid == 0) *zflag = 0;

  const int n = s.n_bus;
  const size_t io = (size_t)b * n;
  // inputs: specified injections and the start point
  for (int i = tid; i < n; i += nt) {
    const int bt = s.bus_type[i];
    const double pg = (kp.pg && bt == 1) ? kp.pg[io + i] : 0.0;
    c.ps[i] = pg - kp.pd[io + i];
    c.qs[i] = -kp.qd[io + i];
    if (kp.mode == MODE_SOLVE) {
      c.vm[i] = bt == 0 ? 1.0 : kp.vset[io + i];
      c.va[i] = 0.0;
    } else {
      c.vm[i] = kp.vm_in[io + i];
      c.va[i] = bt == 2 ? 0.0 : kp.va_in[io + i];
    }
  }
  __syncthreads();
  phase_set_state(s, c, tid, nt);

  const int nb = s.nb;
  int t = 0, status = -1;
  double fn = 0.0;
  const bool mixed = sizeof(T) == 4;
  while (true) {
    int bad = 0;
    fn = phase_mismatch(s, c, tid, nt, &bad);
    if (kp.mode == MODE_EVAL_MISMATCH) { status = 0; break; }
    if (bad) { status = 2; break; }
    if (kp.mode == MODE_SOLVE) {
      if (fn < kp.tol) { status = 0; break; }
      if (t >= kp.max_iter) { status = 1; break; }
    }
    if (kp.mode == MODE_EVAL_FACTOR) {
      status = 0;
      break;
    }
    for (int q = tid; q < 2 * nb; q += nt) c.y[q] = T(-c.F[q]);
    __syncthreads();
    phase_factor<T, LDS>(s, c, tid, nt, kp.gmin, kp.wstride, true, true);
    if (*zflag) { status = 3; break; }
    phase_bsolve(s, c, tid, nt, kp.gmin);
    for (int q = tid; q < 2 * nb; q += nt) c.dx[q] = double(c.y[q]);
    __syncthreads();
    if (mixed) {
      for (int r = 0; r < kp.refine; ++r) {
        phase_dv(s, c, tid, nt);
        phase_residual(s, c, tid, nt);
        phase_fsolve(s, c, tid, nt, kp.gmin);
        phase_bsolve(s, c, tid, nt, kp.gmin);
        for (int q = tid; q < 2 * nb; q += nt) c.dx[q] += double(c.y[q]);
        __syncthreads();
      }
    }
    if (kp.mode == MODE_EVAL_STEP) { status = 0; break; }
    // state update: theta on non-slack buses, |V| on PQ buses
    for (int i = tid; i < n; i += nt) {
      const int a = s.bus_blk[i];
      if (a >= 0) {
        c.va[i] += c.dx[2 * a];
        if (s.bus_type[i] == 0) c.vm[i] += c.dx[2 * a + 1];
      }
    }
    __syncthreads();
    phase_set_state(s, c, tid, nt);
    ++t;
  }

  // outputs
  if (kp.mode == MODE_SOLVE) {
    for (int i = tid; i < n; i += nt) {
      kp.vm_out[io + i] = c.vm[i];
      kp.va_out[io + i] = c.va[i];
    }
    if (tid == 0) {
      if (kp.iters_out) kp.iters_out[b] = t;
      if (kp.status_out) kp.status_out[b] = status;
      if (kp.fnorm_out) kp.fnorm_out[b] = status == 2 ? __builtin_nan("") : fn;
    }
  } else if (kp.mode == MODE_EVAL_MISMATCH || kp.mode == MODE_EVAL_STEP) {
    if (b < kp.count) {
      const double* src = kp.mode == MODE_EVAL_MISMATCH ? c.F : c.dx;
      const int nj = s.nj;
      double* o = kp.out + (size_t)b * nj;
      for (int i = tid; i < n; i += nt) {
        const int a = s.bus_blk[i];
        if (a < 0) continue;
        if (kp.mode == MODE_EVAL_MISMATCH) {
          o[s.ord_p[i]] = src[2 * a];
          if (s.bus_type[i] == 0) o[s.npvpq + s.ord_q[i]] = src[2 * a + 1];
        } else {
          o[s.npq + s.ord_p[i]] = src[2 * a];
          if (s.bus_type[i] == 0) o[s.ord_q[i]] = src[2 * a + 1];
        }
      }
    }
  }
  // keep the converged state and the factors of J1 at it for the adjoint
  const bool keep = (kp.mode == MODE_SOLVE && kp.keep) || kp.mode == MODE_EVAL_FACTOR;
  if (keep && status == 0) {
    phase_factor<T, LDS>(s, c, tid, nt, kp.gmin, kp.wstride, true, false);
    if (*zflag) status = 3;
    if (LDS) {
      T* glu = gt + L.o_lu;
      for (int q = tid; q < 4 * s.nnzb; q += nt) glu[q] = c.lu[q];
      for (int q = tid; q < 4 * nb; q += nt) gt[L.o_dinv + q] = c.dinv[q];
      for (int i = tid; i < n; i += nt) {
        gd[L.o_e + i] = c.e[i]; gd[L.o_f + i] = c.f[i];
        gd[L.o_vm + i] = c.vm[i]; gd[L.o_va + i] = c.va[i];
      }
    }
  }
  if (tid == 0) { gi[0] = keep ? status : -1; gi[1] = t; }
}

// ----------------------------------------------------------------------------
// adjoint kernel (HBM-resident state and factors)

template <typename T>
__global__ void __launch_bounds__(1024) k_adjoint(KParams kp) {
  extern __shared__ __align__(16) unsigned char smem[];
  const DevSym& s = kp.s;
  const int b = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const StateLayout& L = kp.lay;
  double* gd = kp.ws_d + (size_t)b * L.sd;
  T* gt = reinterpret_cast<T*>(kp.ws_t) + (size_t)b * L.st;
  const int* gi = kp.ws_i + (size_t)b * 4;
  Ctx<T> c;
  c.red = reinterpret_cast<double*>(smem);
  c.flags = reinterpret_cast<int*>(smem + kRedBytes);
  bind_state<T>(c, gd, gt, L);
  c.wsp = nullptr;
  const int n = s.n_bus, nb = s.nb;
  const size_t io = (size_t)b * n;
  const bool ok = gi[0] == 0;
  const bool eval = kp.mode == MODE_EVAL_ADJOINT;

  // g_z1 per block: (dL/dtheta, dL/d|V| on PQ) -> kept in F (FP64), y (T)
  if (eval) {
    const double* rhs = kp.rhs + (size_t)b * s.nj;
    for (int i = tid; i < n; i += nt) {
      const int a = s.bus_blk[i];
      if (a < 0) continue;
      const double g0 = rhs[s.npq + s.ord_p[i]];
      const double g1 = s.bus_type[i] == 0 ? rhs[s.ord_q[i]] : 0.0;
      c.F[2 * a] = g0; c.F[2 * a + 1] = g1;
    }
  } else {
    for (int i = tid; i < n; i += nt) {
      const int a = s.bus_blk[i];
      if (a < 0) continue;
      const double g0 = kp.g_va[io + i];
      const double g1 = s.bus_type[i] == 0 ? kp.g_vm[io + i] : 0.0;
      c.F[2 * a] = g0; c.F[2 * a + 1] = g1;
    }
  }
  // I at the kept state (needed by the FP64 transposed products)
  for (int i = tid; i < n; i += nt) {
    double ir = 0.0, ii = 0.0;
    for (int q = s.y_rp[i]; q < s.y_rp[i + 1]; ++q) {
      const int j = s.y_ci[q];
      ir += s.y_g[q] * c.e[j] - s.y_b[q] * c.f[j];
      ii += s.y_g[q] * c.f[j] + s.y_b[q] * c.e[j];
    }
    c.ire[i] = ir; c.iim[i] = ii;
  }
  __syncthreads();
  for (int q = tid; q < 2 * nb; q += nt) c.y[q] = T(c.F[q]);
  __syncthreads();
  phase_ut_solve(s, c, tid, nt, kp.gmin);
  phase_lt_solve(s, c, tid, nt, kp.gmin);
  for (int q = tid; q < 2 * nb; q += nt) c.dx[q] = double(c.y[q]);
  __syncthreads();
  if (sizeof(T) == 4) {
    for (int r = 0; r < kp.refine; ++r) {
      phase_adj_residual(s, c, tid, nt, c.dx, c.F, true);
      phase_ut_solve(s, c, tid, nt, kp.gmin);
      phase_lt_solve(s, c, tid, nt, kp.gmin);
      for (int q = tid; q < 2 * nb; q += nt) c.dx[q] += double(c.y[q]);
      __syncthreads();
    }
  }
  if (eval) {
    if (b < kp.count) {
      double* o = kp.out + (size_t)b * s.nj;
      for (int i = tid; i < n; i += nt) {
        const int a = s.bus_blk[i];
        if (a < 0) continue;
        o[s.ord_p[i]] = c.dx[2 * a];
        if (s.bus_type[i] == 0) o[s.npvpq + s.ord_q[i]] = c.dx[2 * a + 1];
      }
    }
    return;
  }
  // J3^T lam via the transposed product at the solution (-(J3^T lam) lands in aux)
  phase_adj_residual(s, c, tid, nt, c.dx, nullptr, false);
  for (int i = tid; i < n; i += nt) {
    const int a = s.bus_blk[i];
    const int bt = s.bus_type[i];
    double gpd = 0.0, gqd = 0.0, gpg = 0.0, gvs = 0.0;
    if (ok) {
      if (a >= 0) {
        gpd = c.dx[2 * a];
        if (bt == 0) gqd = c.dx[2 * a + 1];
        if (bt == 1) gpg = -c.dx[2 * a];
      }
      if (bt != 0) gvs = kp.g_vm[io + i] + c.aux[i];
    }
    if (kp.g_pd) kp.g_pd[io + i] = gpd;
    if (kp.g_qd) kp.g_qd[io + i] = gqd;
    if (kp.g_pg) kp.g_pg[io + i] = gpg;
    if (kp.g_vset) kp.g_vset[io + i] = gvs;
  }
}

// ----------------------------------------------------------------------------
// dense J1 export in the paper's ordering (evaluation entry point)

__global__ void __launch_bounds__(256) k_jacobian_dense(KParams kp) {
  const DevSym& s = kp.s;
  const int b = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = s.n_bus, nj = s.nj;
  const size_t io = (size_t)b * n;
  double* gd = kp.ws_d + (size_t)b * kp.lay.sd;
  double *e = gd + kp.lay.o_e, *f = gd + kp.lay.o_f, *vm = gd + kp.lay.o_vm;
  double *ire = gd + kp.lay.o_ire, *iim = gd + kp.lay.o_iim;
  for (int i = tid; i < n; i += nt) {
    vm[i] = kp.vm_in[io + i];
    const double va = s.bus_type[i] == 2 ? 0.0 : kp.va_in[io + i];
    e[i] = vm[i] * cos(va);
    f[i] = vm[i] * sin(va);
  }
  __syncthreads();
  for (int i = tid; i < n; i += nt) {
    double ir = 0.0, ii = 0.0;
    for (int q = s.y_rp[i]; q < s.y_rp[i + 1]; ++q) {
      const int j = s.y_ci[q];
      ir += s.y_g[q] * e[j] - s.y_b[q] * f[j];
      ii += s.y_g[q] * f[j] + s.y_b[q] * e[j];
    }
    ire[i] = ir; iim[i] = ii;
  }
  __syncthreads();
  double* o = kp.out + (size_t)b * nj * nj;
  for (size_t q = tid; q < (size_t)nj * nj; q += nt) o[q] = 0.0;
  __syncthreads();
  for (int i = tid; i < n; i += nt) {
    if (s.bus_type[i] == 2) continue;
    const int rP = s.ord_p[i];
    const int rQ = s.bus_type[i] == 0 ? s.npvpq + s.ord_q[i] : -1;
    for (int q = s.y_rp[i]; q < s.y_rp[i + 1]; ++q) {
      const int m = s.y_ci[q];
      if (s.bus_type[m] == 2) continue;
      const B4d x = jac_entries(i, m, s.y_g[q], s.y_b[q], e, f, vm, ire, iim);
      const int cT = s.npq + s.ord_p[m];
      const int cV = s.bus_type[m] == 0 ? s.ord_q[m] : -1;
      o[(size_t)rP * nj + cT] = x.v[0];
      if (cV >= 0) o[(size_t)rP * nj + cV] = x.v[1];
      if (rQ >= 0) {
        o[(size_t)rQ * nj + cT] = x.v[2];
        if (cV >= 0) o[(size_t)rQ * nj + cV] = x.v[3];
      }
    }
  }
}

// ----------------------------------------------------------------------------
// launchers

template <typename T>
static hipError_t launch_newton_t(const KParams& kp, int grid, int nt, size_t lds, bool lds_res,
                                  hipStream_t st) {
  if (lds_res) {
    hipLaunchKernelGGL((k_newton<T, true>), dim3(grid), dim3(nt), lds, st, kp);
  } else {
    hipLaunchKernelGGL((k_newton<T, false>), dim3(grid), dim3(nt), lds, st, kp);
  }
  return hipGetLastError();
}

hipError_t launch_newton(const KParams& kp, bool fp32, int grid, int nt, size_t lds, bool lds_res,
                         hipStream_t st) {
  return fp32 ? launch_newton_t<float>(kp, grid, nt, lds, lds_res, st)
              : launch_newton_t<double>(kp, grid, nt, lds, lds_res, st);
}

hipError_t launch_adjoint(const KParams& kp, bool fp32, int grid, int nt, hipStream_t st) {
  const size_t lds = kScratchBytes;
  if (fp32) {
    hipLaunchKernelGGL((k_adjoint<float>), dim3(grid), dim3(nt), lds, st, kp);
  } else {
    hipLaunchKernelGGL((k_adjoint<double>), dim3(grid), dim3(nt), lds, st, kp);
  }
  return hipGetLastError();
}

hipError_t launch_jacobian_dense(const KParams& kp, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobian_dense, dim3(grid), dim3(256), 0, st, kp);
  return hipGetLastError();
}

hipError_t set_lds_limits(size_t max_lds) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* fn) {
    hipError_t r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
    if (r != hipSuccess) e = r;
  };
  set(reinterpret_cast<const void*>(&k_newton<double, true>));
  set(reinterpret_cast<const void*>(&k_newton<double, false>));
  set(reinterpret_cast<const void*>(&k_newton<float, true>));
  set(reinterpret_cast<const void*>(&k_newton<float, false>));
  return e;
}

}  // namespace sable
