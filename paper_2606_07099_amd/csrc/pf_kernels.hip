// Device kernels of the batched Newton power flow for CDNA4 (gfx950).
//
// One workgroup owns a slice of S scenarios (S = 1, 2, 4 or 8) for the whole
// Newton solve, with no host round trip per iteration: complex Y_bus SpMV +
// mismatch, per-scenario convergence test, Jacobian value evaluation
// (Algorithm 1) into the fixed symbolic pattern, a 2x2-block LU
// refactorisation scheduled right-looking by levels (forward solve fused),
// the level-scheduled backward solve, FP64-residual refinement in the
// mixed-precision mode, and the state update.  Converged scenarios of a slice
// freeze while the others continue.
//
// Two residency modes:
//  * LDS-resident (small grids): the symbolic image and the whole state of
//    the S scenarios live in LDS; arrays are interleaved by scenario, so a
//    lane's scenario index is its lane index modulo S and the S lanes that
//    share an index load or update adjacent LDS words.
//  * HBM-resident (large grids, S = 1): the state lives in the scenario's
//    HBM workspace, the symbolic arrays are read from the shared image (L2),
//    and only the factor row under elimination is staged in LDS.
#include "pf_kernels.h"

#include <hip/hip_runtime.h>

namespace sable {

// ----------------------------------------------------------------------------
// per-phase wall-clock accounting, compiled in with -DSABLE_PHASE_CLOCKS:
// thread 0 of workgroup 0 adds the ticks of the constant-rate wall clock
// between consecutive phase marks to one counter per phase (every mark
// follows a workgroup barrier, so the interval is the workgroup's time in
// that phase).  Without the flag the marks compile to nothing.

#ifdef SABLE_PHASE_CLOCKS
__device__ unsigned long long g_phase_ticks[kPhaseSlots];
struct PhaseClock {
  bool on;
  unsigned long long t0;
  __device__ __forceinline__ explicit PhaseClock(int tid) : on(tid == 0 && blockIdx.x == 0), t0(0) {
    if (on) t0 = wall_clock64();
  }
  __device__ __forceinline__ void mark(int ph) {
    if (on) {
      const unsigned long long t = wall_clock64();
      g_phase_ticks[ph] += t - t0;
      t0 = t;
    }
  }
  __device__ __forceinline__ void count(int slot) {
    if (on) g_phase_ticks[slot] += 1;
  }
};
#else
struct PhaseClock {
  __device__ __forceinline__ explicit PhaseClock(int) {}
  __device__ __forceinline__ void mark(int) {}
  __device__ __forceinline__ void count(int) {}
};
#endif

// ----------------------------------------------------------------------------
// small helpers

template <typename T>
struct Blk { T a, b, c, d; };  // row-major 2x2 block [[a, b], [c, d]]

// every block (factors, pivot inverses, the LDS tail copy) starts 16-byte
// aligned in every layout, so a block moves in 16-byte vector operations
__device__ __forceinline__ Blk<float> ld_blk(const float* p) {
  using V = float __attribute__((ext_vector_type(4)));
  const V v = *reinterpret_cast<const V*>(__builtin_assume_aligned(p, 16));
  return {v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ Blk<double> ld_blk(const double* p) {
  using V = double __attribute__((ext_vector_type(2)));
  const V* q = reinterpret_cast<const V*>(__builtin_assume_aligned(p, 16));
  const V u = q[0], v = q[1];
  return {u.x, u.y, v.x, v.y};
}
__device__ __forceinline__ void st_blk(float* p, const Blk<float>& x) {
  using V = float __attribute__((ext_vector_type(4)));
  *reinterpret_cast<V*>(__builtin_assume_aligned(p, 16)) = V{x.a, x.b, x.c, x.d};
}
__device__ __forceinline__ void st_blk(double* p, const Blk<double>& x) {
  using V = double __attribute__((ext_vector_type(2)));
  V* q = reinterpret_cast<V*>(__builtin_assume_aligned(p, 16));
  q[0] = V{x.a, x.b};
  q[1] = V{x.c, x.d};
}
// streaming block load: HBM values read once per pass, marked non-temporal
// so that they do not displace the gathered unknowns from the caches
__device__ __forceinline__ Blk<float> ld_blk_nt(const float* p) {
  using V = float __attribute__((ext_vector_type(4)));
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(__builtin_assume_aligned(p, 16)));
  return {v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ Blk<double> ld_blk_nt(const double* p) {
  using V = double __attribute__((ext_vector_type(2)));
  const V* q = reinterpret_cast<const V*>(__builtin_assume_aligned(p, 16));
  const V u = __builtin_nontemporal_load(q), v = __builtin_nontemporal_load(q + 1);
  return {u.x, u.y, v.x, v.y};
}

template <typename T>
__device__ __forceinline__ Blk<T> mul(const Blk<T>& x, const Blk<T>& y) {
  return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}

// reciprocal of a pivot determinant: the hardware reciprocal (1 ulp) for
// FP32 factors, which the FP64 residual of the Newton loop corrects; an
// exact division for FP64 factors
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// interleaved indexing inside a slice of S scenarios
template <int S> __device__ __forceinline__ int sI(int i, int s) { return i * S + s; }
template <int S> __device__ __forceinline__ int sP(int a, int s) { return (a * S + s) * 2; }
template <int S> __device__ __forceinline__ int sB(int p, int s) { return (p * S + s) * 4; }

// symbolic arrays, bound to LDS or to the device image
struct Sym {
  const int *bus_type, *bus_blk, *y_rp, *y_ci;
  const double *y_g, *y_b;
  const int *rp, *ci, *diag;
  const int4* fill4;
  const int *tail_pos, *tail_split, *tail_prog;
  const unsigned* tail_mask;
  const int *y_tr, *ord_p, *ord_q;
  const int *f_ptr, *f_blob, *fs_ptr, *fs_blob, *bs_ptr, *bs_blob;
  const int* tail_cblk;
};

__device__ __forceinline__ Sym bind_sym(const unsigned char* nb, const unsigned char* g,
                                        const SymOffsets& o) {
  Sym m;
  auto I = [](const unsigned char* b, int off) { return reinterpret_cast<const int*>(b + off); };
  m.bus_type = I(nb, o.bus_type);
  m.bus_blk = I(nb, o.bus_blk);
  m.y_rp = I(nb, o.y_rp);
  m.y_ci = I(nb, o.y_ci);
  m.y_g = reinterpret_cast<const double*>(nb + o.y_g);
  m.y_b = reinterpret_cast<const double*>(nb + o.y_b);
  m.rp = I(nb, o.rp);
  m.ci = I(nb, o.ci);
  m.diag = I(nb, o.diag);
  m.fill4 = reinterpret_cast<const int4*>(nb + o.fill4);
  m.tail_pos = I(nb, o.tail_pos);
  m.tail_split = I(nb, o.tail_split);
  m.tail_mask = reinterpret_cast<const unsigned*>(nb + o.tail_mask);
  m.f_ptr = I(nb, o.f_ptr);
  m.f_blob = I(nb, o.f_blob);
  m.fs_ptr = I(nb, o.fs_ptr);
  m.fs_blob = I(nb, o.fs_blob);
  m.bs_ptr = I(nb, o.bs_ptr);
  m.bs_blob = I(nb, o.bs_blob);
  m.tail_prog = I(g, o.tail_prog);
  m.y_tr = I(g, o.y_tr);   // LDS-resident adjoint slices rebind it to their LDS copy
  m.ord_p = I(g, o.ord_p);
  m.ord_q = I(g, o.ord_q);
  m.tail_cblk = I(g, o.tail_cblk);
  return m;
}

// per-slice state; element k of scenario s sits at k*S + s
// per-slice state.  e f |V| 1/|V| I_re I_im dV_re dV_im of bus i, scenario s
// sit at index i * gs + s of their arrays (g(i, s) below): gs = S when every
// array is interleaved on its own (LDS-resident slices), 8 S when a bus's eight
// values are grouped (HBM-resident slices: a gather of one bus then touches
// one 64-byte run per scenario instead of one per value).  The other arrays
// are interleaved by scenario: element k of scenario s at k * S + s.
template <typename T>
struct St {
  double *e, *f, *vm, *va, *ire, *iim, *ps, *qs, *dvr, *dvi, *aux, *rvm, *F, *dx;
  T *y, *lu, *dinv;
  int gs;
  __device__ __forceinline__ int g(int i, int s) const { return i * gs + s; }
};

template <typename T, int S>
__device__ __forceinline__ St<T> bind_state(double* d, T* t, const StateLayout& L) {
  St<T> c;
  c.e = d + L.o_e * S; c.f = d + L.o_f * S; c.vm = d + L.o_vm * S; c.va = d + L.o_va * S;
  c.ire = d + L.o_ire * S; c.iim = d + L.o_iim * S; c.ps = d + L.o_ps * S; c.qs = d + L.o_qs * S;
  c.dvr = d + L.o_dvr * S; c.dvi = d + L.o_dvi * S; c.aux = d + L.o_aux * S; c.rvm = d + L.o_rvm * S;
  c.F = d + L.o_F * S; c.dx = d + L.o_dx * S;
  c.y = t + L.o_y * S; c.lu = t + L.o_lu * S; c.dinv = t + L.o_dinv * S;
  c.gs = L.gk * S;
  return c;
}

// Jacobian entries of J1 = dF1/dz1 for the bus pair (i, m): rows (dP_i, dQ_i),
// columns (theta_m, |V|_m), in rectangular coordinates V = e + jf, I = Y V.
// For i != m the products |V_i||V_m| cos(theta_im) = e_i e_m + f_i f_m and
// |V_i||V_m| sin(theta_im) = f_i e_m - e_i f_m replace the trigonometric
// terms; the values equal the closed forms of Algorithm 1.
struct J4 { double v[4]; };

// (rv = 1 / |V| of the bus whose magnitude is the column unknown)
__device__ __forceinline__ J4 jac_diag(double G, double B, double ei, double fi, double vmi, double rvi,
                                       double iri, double iii) {
  const double P = ei * iri + fi * iii;
  const double Q = fi * iri - ei * iii;
  const double v2 = vmi * vmi;
  return {{Q + B * v2, -P * rvi - G * vmi, -P + G * v2, -Q * rvi + B * vmi}};
}

__device__ __forceinline__ J4 jac_off(double G, double B, double ei, double fi, double em, double fm,
                                      double rvm) {
  const double cc = ei * em + fi * fm;
  const double ss = fi * em - ei * fm;
  const double gs_bc = G * ss - B * cc;
  const double gc_bs = G * cc + B * ss;
  return {{-gs_bc, -gc_bs * rvm, gc_bs, -gs_bc * rvm}};
}

// The 2x2 block of the padded block system at LU position p for scenario s.
// PV buses keep a dummy |V| unknown and a dummy dQ row: identity on the
// diagonal, zero coupling; fill-in positions start at zero.  Split into the
// gathers (fill record, then the Y entry and the two buses' state) and the
// arithmetic, so that several blocks' gathers are in flight together.
struct FillIn {
  int4 r;           // Y entry, row bus, column bus, flags
  double g, b;      // Y entry
  double x[6];      // diagonal: e f |V| 1/|V| I_re I_im of the bus; else e f of the row bus, e f 1/|V| of the column bus
};

template <typename T, int S, bool RES>
__device__ __forceinline__ void fill_gather(const Sym& m, const St<T>& c, int s, FillIn& q) {
  const int4 r = q.r;
  const bool dg = r.w & 1;
  q.g = r.x < 0 ? 0.0 : m.y_g[r.x];
  q.b = r.x < 0 ? 0.0 : m.y_b[r.x];
  const int is = c.g(r.y, s), ms = c.g(r.z, s);
  // one-scenario slices skip the gathers of fill-in positions (no value);
  // in wider slices the masked loads cost more than the lines they save
  const bool fill_in = !RES && S == 1 && r.x < 0 && !dg;
  q.x[0] = fill_in ? 0.0 : c.e[is];
  q.x[1] = fill_in ? 0.0 : c.f[is];
  if (dg) {
    // (with the state in HBM |V| and 1/|V| are formed from e and f, below)
    q.x[2] = RES ? c.vm[is] : 0.0;
    q.x[3] = RES ? c.rvm[is] : 0.0;
    q.x[4] = c.ire[is];
    q.x[5] = c.iim[is];
  } else {
    q.x[2] = fill_in ? 0.0 : c.e[ms];
    q.x[3] = fill_in ? 0.0 : c.f[ms];
    // with the state in HBM the column bus's 1/|V| is formed from its e and
    // f (hardware estimate and two Newton steps) instead of gathering a third
    // value per block (in LDS the gather is the cheaper)
    q.x[4] = RES ? c.rvm[ms] : 0.0;
    q.x[5] = 0.0;
  }
}

// 1/sqrt(x) for x > 0 to a few units in the last place: the hardware
// estimate refined by two Newton steps
// sin and cos of an FP64 angle behind a call boundary: inlined into the
// 1024-thread Newton kernel (128 registers per lane), the polynomial's
// constants were hoisted to the kernel's start, spilled, and reloaded one by
// one from scratch for every item of the state update; inside a call they are
// formed where they are used (one value reloaded per item instead of nine)
__device__ __attribute__((noinline)) double2 sincos_call(double x) {
  double sn, cs;
  sincos(x, &sn, &cs);
  return make_double2(sn, cs);
}

__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

template <typename T, bool RES>
__device__ __forceinline__ Blk<T> fill_value(FillIn q) {
  const int4 r = q.r;
  const bool dg = r.w & 1;
  if (r.x < 0 && !dg) return {T(0), T(0), T(0), T(0)};
  if (!RES && !dg) q.x[4] = rsqrt_nr(q.x[2] * q.x[2] + q.x[3] * q.x[3]);
  if (!RES && dg) {
    const double v2 = q.x[0] * q.x[0] + q.x[1] * q.x[1];
    q.x[3] = rsqrt_nr(v2);
    q.x[2] = v2 * q.x[3];
  }
  J4 x = dg ? jac_diag(q.g, q.b, q.x[0], q.x[1], q.x[2], q.x[3], q.x[4], q.x[5])
            : jac_off(q.g, q.b, q.x[0], q.x[1], q.x[2], q.x[3], q.x[4]);
  if (r.w & 2) { x.v[2] = 0.0; x.v[3] = 0.0; }
  if (r.w & 4) { x.v[1] = 0.0; x.v[3] = 0.0; }
  if ((r.w & 3) == 3) x.v[3] = 1.0;
  return {T(x.v[0]), T(x.v[1]), T(x.v[2]), T(x.v[3])};
}

// lanes per row group: enough groups for the rows of a level, at least S
// lanes (one per scenario of the slice), at least gmin (HBM workspace limit)
__device__ __forceinline__ int pick_group(int nrows, int nt, int gmin) {
  int g = 64;
  while (g > gmin && (nt / g) < nrows) g >>= 1;
  return g;
}

// group geometry for G lanes per item (G a power of two)
struct Grp {
  int G, gid, lane, ng;
};
__device__ __forceinline__ Grp groups(int nitems, int tid, int nt, int gmin) {
  const int G = pick_group(nitems, nt, gmin);
  const int lg = __builtin_ctz(G);
  return {G, tid >> lg, tid & (G - 1), nt >> lg};
}

// value of lane (this lane xor O): partners within a 16-lane row move by DPP
// (a VALU operation: quad permutations for O = 1, 2; a row shift left or
// right, picked per lane, for O = 4, 8), farther partners by ds_bpermute
template <int O>
__device__ __forceinline__ int xor_lane(int v) {
  if constexpr (O == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  else if constexpr (O == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  else if constexpr (O == 4 || O == 8) {
    const int up = __builtin_amdgcn_mov_dpp(v, 0x100 | O, 0xF, 0xF, false);     // row_shl: lane + O
    const int down = __builtin_amdgcn_mov_dpp(v, 0x110 | O, 0xF, 0xF, false);   // row_shr: lane - O
    return (__lane_id() & O) ? down : up;
  } else {
    return __shfl_xor(v, O);
  }
}
template <int O>
__device__ __forceinline__ float xor_lane(float v) {
  return __int_as_float(xor_lane<O>(__float_as_int(v)));
}
template <int O>
__device__ __forceinline__ double xor_lane(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = xor_lane<O>((int)(b & 0xffffffffll)), hi = xor_lane<O>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over the G/S entry lanes of one scenario inside a group (G a power of
// two, groups aligned to G lanes, every lane of a group active)
template <typename T, int S>
__device__ __forceinline__ T group_sum(T v, int G) {
  if (G > 32 && S <= 32) v += xor_lane<32>(v);
  if (G > 16 && S <= 16) v += xor_lane<16>(v);
  if (G > 8 && S <= 8) v += xor_lane<8>(v);
  if (G > 4 && S <= 4) v += xor_lane<4>(v);
  if (G > 2 && S <= 2) v += xor_lane<2>(v);
  if (G > 1 && S <= 1) v += xor_lane<1>(v);
  return v;
}

// per-scenario max over the workgroup of v and OR of bad (a thread's scenario
// is tid % S); results land in the scratch arrays fn[S] / bad[S]
template <int S>
__device__ __forceinline__ void block_max(double v, int bad, unsigned char* scr, int tid, int nt) {
  double* red = reinterpret_cast<double*>(scr + kRedOff);
  int* flg = reinterpret_cast<int*>(scr + kFlagOff);
  if (S <= 32) { v = fmax(v, xor_lane<32>(v)); bad |= xor_lane<32>(bad); }
  if (S <= 16) { v = fmax(v, xor_lane<16>(v)); bad |= xor_lane<16>(bad); }
  if (S <= 8) { v = fmax(v, xor_lane<8>(v)); bad |= xor_lane<8>(bad); }
  if (S <= 4) { v = fmax(v, xor_lane<4>(v)); bad |= xor_lane<4>(bad); }
  if (S <= 2) { v = fmax(v, xor_lane<2>(v)); bad |= xor_lane<2>(bad); }
  if (S <= 1) { v = fmax(v, xor_lane<1>(v)); bad |= xor_lane<1>(bad); }
  const int w = tid >> 6, l = tid & 63;
  if (l < S) { red[w * S + l] = v; flg[w * S + l] = bad; }
  __syncthreads();
  if (tid < S) {
    double mx = 0.0;
    int b = 0;
    for (int k = 0; k < (nt >> 6); ++k) { mx = fmax(mx, red[k * S + tid]); b |= flg[k * S + tid]; }
    reinterpret_cast<double*>(scr + kFnOff)[tid] = mx;
    reinterpret_cast<int*>(scr + kBadOff)[tid] = b;
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// phases (each ends with a workgroup barrier)

// The bus-indexed passes (mismatch, refinement dV and residual) give each
// thread two items (bus, scenario) at a time, nt apart (so both belong to the
// same scenario), and issue each item's own loads before its Y_bus row
// product: with the state in HBM every load is a round trip, and a loop that
// waits for one row entry at a time leaves the memory system idle.

// Y_bus row products I = sum_q Y_iq (xr + j xi)_j of two items at once: four
// entries of each row per round, every index, admittance and gathered value
// of the round loaded before the arithmetic.  Entries past a row's end load
// bus 0 (in bounds) and are not added; each row is summed in column order.
template <int S, int U, int W>
__device__ __forceinline__ void yrow_multi(const Sym& m, const double* xr, const double* xi, int gs,
                                           const int (&i)[U], int s, const bool (&v)[U], double (&ar)[U],
                                           double (&ai)[U]) {
  int q[U], q1[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    q[u] = v[u] ? m.y_rp[i[u]] : 0;
    q1[u] = v[u] ? m.y_rp[i[u] + 1] : 0;
    ar[u] = 0.0;
    ai[u] = 0.0;
  }
  while (true) {
    bool more = false;
#pragma unroll
    for (int u = 0; u < U; ++u) more |= q[u] < q1[u];
    if (!more) break;
    int j[U][W];
    double g[U][W], b[U][W], x[U][W], y[U][W];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const bool in = q[u] + w < q1[u];
        j[u][w] = in ? m.y_ci[q[u] + w] : 0;
        g[u][w] = in ? m.y_g[q[u] + w] : 0.0;
        b[u][w] = in ? m.y_b[q[u] + w] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int w = 0; w < W; ++w) {
        x[u][w] = xr[j[u][w] * gs + s];
        y[u][w] = xi[j[u][w] * gs + s];
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int w = 0; w < W; ++w)
        if (q[u] + w < q1[u]) {
          ar[u] += g[u][w] * x[u][w] - b[u][w] * y[u][w];
          ai[u] += g[u][w] * y[u][w] + b[u][w] * x[u][w];
        }
      q[u] += W;
    }
  }
}

// items per thread and row entries per round of the bus-indexed passes
constexpr int kBusU = 1, kBusW = 4;

// I = Y V, S = V conj(I), F1 = spec - calc of every bus (F indexed by bus,
// two entries each: dP, and dQ on PQ buses); ||F1||_inf per scenario.  The
// Newton step's right-hand side y = -F1 goes to the block rows as well.
template <typename T, int S>
__device__ __forceinline__ void phase_mismatch(const Sym& m, const Dims& D, St<T>& c, int tid, int nt,
                               unsigned char* scr) {
  double mx = 0.0;
  int bad = 0;
  const int s = tid % S, N = D.n_bus * S;
  for (int base = tid; base < N; base += kBusU * nt) {
    int i[kBusU], a[kBusU], bt[kBusU];
    bool v[kBusU];
    double ei[kBusU], fi[kBusU], ps[kBusU], qs[kBusU];
#pragma unroll
    for (int u = 0; u < kBusU; ++u) {
      const int idx = base + u * nt;
      v[u] = idx < N;
      i[u] = v[u] ? idx / S : 0;
      a[u] = m.bus_blk[i[u]];
      bt[u] = m.bus_type[i[u]];
      const int o = v[u] ? idx : base;
      const int go = c.g(i[u], s);
      ei[u] = c.e[go];
      fi[u] = c.f[go];
      ps[u] = c.ps[o];
      qs[u] = c.qs[o];
    }
    double ir[kBusU], ii[kBusU];
    yrow_multi<S, kBusU, kBusW>(m, c.e, c.f, c.gs, i, s, v, ir, ii);
#pragma unroll
    for (int u = 0; u < kBusU; ++u) {
      if (!v[u]) continue;
      const int go = c.g(i[u], s);
      c.ire[go] = ir[u];
      c.iim[go] = ii[u];
      if (a[u] >= 0) {
        const double P = ei[u] * ir[u] + fi[u] * ii[u];
        const double Q = fi[u] * ir[u] - ei[u] * ii[u];
        const double F0 = ps[u] - P;
        const double F1 = bt[u] == 0 ? qs[u] - Q : 0.0;
        c.F[sP<S>(i[u], s)] = F0;
        c.F[sP<S>(i[u], s) + 1] = F1;
        c.y[sP<S>(a[u], s)] = T(-F0);
        c.y[sP<S>(a[u], s) + 1] = T(-F1);
        bad |= !(isfinite(F0) && isfinite(F1));
        mx = fmax(mx, fmax(fabs(F0), fabs(F1)));
      }
    }
  }
  __syncthreads();
  block_max<S>(mx, bad, scr, tid, nt);
}

// the same pass for LDS-resident FP64 slices: one bus per thread, its row of
// Y_bus walked entry by entry (with the FP64 factors' register budget this
// form issues fewer instructions than the rounds of four entries)
template <typename T, int S>
__device__ __forceinline__ void phase_mismatch_lds(const Sym& m, const Dims& D, St<T>& c, int tid, int nt,
                                                   unsigned char* scr) {
  double mx = 0.0;
  int bad = 0;
  for (int idx = tid; idx < D.n_bus * S; idx += nt) {
    const int i = idx / S, s = idx % S;
    double ir = 0.0, ii = 0.0;
    for (int q = m.y_rp[i]; q < m.y_rp[i + 1]; ++q) {
      const int j = c.g(m.y_ci[q], s);
      const double g = m.y_g[q], b = m.y_b[q];
      ir += g * c.e[j] - b * c.f[j];
      ii += g * c.f[j] + b * c.e[j];
    }
    const int go = c.g(i, s);
    c.ire[go] = ir;
    c.iim[go] = ii;
    const int a = m.bus_blk[i];
    if (a >= 0) {
      const double ei = c.e[go], fi = c.f[go];
      const double P = ei * ir + fi * ii;
      const double Q = fi * ir - ei * ii;
      const double F0 = c.ps[idx] - P;
      const double F1 = m.bus_type[i] == 0 ? c.qs[idx] - Q : 0.0;
      c.F[sP<S>(i, s)] = F0;
      c.F[sP<S>(i, s) + 1] = F1;
      c.y[sP<S>(a, s)] = T(-F0);
      c.y[sP<S>(a, s) + 1] = T(-F1);
      bad |= !(isfinite(F0) && isfinite(F1));
      mx = fmax(mx, fmax(fabs(F0), fabs(F1)));
    }
  }
  __syncthreads();
  block_max<S>(mx, bad, scr, tid, nt);
}

// orders this wavefront's earlier global stores before its later loads (HBM
// state); LDS operations of a wavefront are already in order
template <bool RES>
__device__ __forceinline__ void wave_order() {
  if (!RES) __threadfence_block();
}

// Jacobian values of every block of the pattern (fill-in blocks zeroed) for
// the S scenarios: independent work, one pass before the factorisation.
template <typename T, int S, bool RES>
__device__ __forceinline__ void phase_fill(const Sym& m, const Dims& D, St<T>& c, int tid, int nt) {
  constexpr int NB = RES ? 4 : 2;
  // NB blocks per thread have their gathers in flight together
  const int N = D.nnzb * S;
  for (int base = tid; base < N; base += NB * nt) {
    FillIn q[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = base + u * nt;
      q[u].r = idx < N ? m.fill4[idx / S] : make_int4(-1, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) fill_gather<T, S, RES>(m, c, (base + u * nt) % S, q[u]);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int idx = base + u * nt;
      if (idx < N) st_blk(c.lu + sB<S>(idx / S, idx % S), fill_value<T, RES>(q[u]));
    }
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// level-scheduled factor and solves.  HBM-resident slices first copy each
// chunk of level metadata (tasks, steps, targets / rows, columns) into LDS
// with the whole workgroup, so that only the value loads of a step reach HBM

// The metadata chunks of a schedule, pass after pass: in place when the
// image is LDS-resident, else copied into LDS by the whole workgroup.  The
// copy of the next chunk is started before the current one is processed: its
// first 16 bytes per lane are loaded into registers right after the chunk's
// barrier, so their HBM/L2 latency overlaps the pass, and written to LDS at
// the start of the next pass (the rest of a chunk larger than one int4 per
// lane is copied there directly).
template <bool STAGE>
struct ChunkStager {
  const int* ptr;
  const int* blob;
  int4* lds;
  int tid, nt, nch;
  int4 pre;     // this lane's first int4 of the next chunk
  int b0, n4;   // the next chunk: start (int32 words) and length (int4)

  __device__ __forceinline__ ChunkStager(const int* ptr_, const int* blob_, int nch_, unsigned char* lds_,
                                         int tid_, int nt_)
      : ptr(ptr_), blob(blob_), lds(reinterpret_cast<int4*>(lds_)), tid(tid_), nt(nt_), nch(nch_),
        pre(make_int4(0, 0, 0, 0)), b0(0), n4(0) {
    if (STAGE && nch > 0) fetch(0);
  }
  __device__ __forceinline__ void fetch(int c) {
    b0 = ptr[c];
    n4 = (ptr[c + 1] - b0) >> 2;
    if (tid < n4) pre = reinterpret_cast<const int4*>(blob + b0)[tid];
  }
  // chunk c (in order c = 0, 1, ...): its base in LDS or in the image
  __device__ __forceinline__ const int* get(int c) {
    if (!STAGE) return blob + ptr[c];
    const int4* src = reinterpret_cast<const int4*>(blob + b0);
    if (tid < n4) lds[tid] = pre;
    for (int q = tid + nt; q < n4; q += nt) lds[q] = src[q];
    __syncthreads();
    if (c + 1 < nch) fetch(c + 1);
    return reinterpret_cast<const int*>(lds);
  }
};

// Block LU (unit block-lower L, block-upper U with full 2x2 pivots) on the
// fixed pattern, right-looking by levels with owner-computes rows: at level h
// every row with a pivot k finished at level h-1 applies
//   L_ak = A_ak U_kk^-1,  A_aj -= L_ak U_kj  (j in U(k,>k)),  y_a -= L_ak y_k
// (the last term is the fused forward solve), and a row whose last pivot is
// in inverts its own pivot block.  A row's entry A_ak is final when step k
// runs because every pivot that updates it sits at a lower level.  The G
// lanes of a task share one row (lane = scenario + S * entry) and belong to
// one wavefront: LDS operations of a wavefront complete in program order;
// in HBM a fence orders successive steps unless one lane per scenario owns
// the task (then every target is written and re-read by that lane).  The
// level metadata comes in chunks of whole rows (RES: in place in the LDS
// image; else staged into LDS).
template <typename T, int S, bool RES>
__device__ __forceinline__ void phase_factor(const Sym& m, const Dims& D, St<T>& c, int tid, int nt, int gmin,
                                             bool fwd, int* piv, unsigned char* lds) {
  ChunkStager<!RES> stg(m.f_ptr, m.f_blob, D.nch_f, lds, tid, nt);
  for (int ch = 0; ch < D.nch_f; ++ch) {
    const int* h = stg.get(ch);
    const int ntask = h[0], nstep = h[1];
    const int4* tk4 = reinterpret_cast<const int4*>(h + 4);
    const int4* st4 = tk4 + ntask + 1;
    const int* tg = reinterpret_cast<const int*>(st4 + nstep + 1);
    const Grp g = groups(ntask, tid, nt, gmin);
    const int s = g.lane % S, e = g.lane / S, E = g.G / S;
    for (int ti = g.gid; ti < ntask; ti += g.ng) {
      const int4 tk = tk4[ti];   // row, rp[row], pivot-block offset or -1, first step
      const int a = tk.x, se = tk4[ti + 1].w;
      T* W = c.lu + sB<S>(tk.y, 0);
      T y0 = T(0), y1 = T(0);
      if (fwd) { y0 = c.y[sP<S>(a, s)]; y1 = c.y[sP<S>(a, s) + 1]; }
      for (int i = tk.w; i < se; ++i) {
        if (i > tk.w && E > 1) wave_order<RES>();   // the previous step's targets may feed this one
        const int4 st = st4[i];   // q, k, first U position, first target
        const int n = st4[i + 1].w - st.w;
        const int k = st.y;
        const Blk<T> L = mul(ld_blk(W + sB<S>(st.x, s)), ld_blk(c.dinv + sB<S>(k, s)));
        if (fwd) {
          const T yk0 = c.y[sP<S>(k, s)], yk1 = c.y[sP<S>(k, s) + 1];
          y0 -= L.a * yk0 + L.b * yk1;
          y1 -= L.c * yk0 + L.d * yk1;
        }
        constexpr int NB = 2;   // the targets of one step are distinct: loads first
        int t = e;
        for (; t + (NB - 1) * E < n; t += NB * E) {
          Blk<T> U[NB], x[NB];
          T* w[NB];
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            U[u] = ld_blk(c.lu + sB<S>(st.z + t + u * E, s));
            w[u] = W + sB<S>(tg[st.w + t + u * E], s);
            x[u] = ld_blk(w[u]);
          }
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            const Blk<T> LU = mul(L, U[u]);
            x[u].a -= LU.a; x[u].b -= LU.b; x[u].c -= LU.c; x[u].d -= LU.d;
            st_blk(w[u], x[u]);
          }
        }
        for (; t < n; t += E) {
          const Blk<T> U = ld_blk(c.lu + sB<S>(st.z + t, s));
          T* w = W + sB<S>(tg[st.w + t], s);
          Blk<T> x = ld_blk(w);
          const Blk<T> LU = mul(L, U);
          x.a -= LU.a; x.b -= LU.b; x.c -= LU.c; x.d -= LU.d;
          st_blk(w, x);
        }
        if (e == 0) st_blk(W + sB<S>(st.x, s), L);
      }
      if (e == 0) {
        if (tk.z >= 0) {
          // a task that inverts its row's pivot block eliminates only
          // children of the row in the elimination tree, whose first U
          // column is the row itself: the diagonal is target 0 of every
          // step, updated by this lane, so only the other lanes' targets of
          // earlier steps (several steps) need the fence before it is read
          if (se - tk.w > 1 && E > 1) wave_order<RES>();
          const Blk<T> Dk = ld_blk(W + sB<S>(tk.z, s));
          const T det = Dk.a * Dk.d - Dk.b * Dk.c;
          const T inv = recip(det);
          const Blk<T> Di = {Dk.d * inv, -Dk.b * inv, -Dk.c * inv, Dk.a * inv};
          const T eps = sizeof(T) == 8 ? T(1e-14) : T(1e-7);
          const bool zero = !(fabs(Dk.a) > eps * (fabs(Dk.a) + fabs(Dk.b))) ||
                            !(fabs(det) > eps * fabs(Dk.a) * (fabs(Dk.c) + fabs(Dk.d))) ||
                            !isfinite(inv);
          if (zero) piv[s] = 1;
          st_blk(c.dinv + sB<S>(a, s), Di);
        }
        if (fwd) { c.y[sP<S>(a, s)] = y0; c.y[sP<S>(a, s) + 1] = y1; }
      }
    }
    __syncthreads();
  }
}

// level-scheduled row solves of the rows outside the dense tail, rows and
// their columns from the metadata chunks: forward (unit block-lower L, in
// place in y) or backward (U with the inverted pivot blocks)
// The backward pass can also hand its result to the FP64 correction of the
// scenarios in `mask`: dxmode 1 sets dx = y, dxmode 2 adds y to dx (each row
// is written once, by its lane of entry 0, so no separate copy pass is needed).
template <typename T, int S, bool RES, bool LOWER>
__device__ __forceinline__ void phase_solve(const Sym& m, const Dims& D, St<T>& c, int tid, int nt, int gmin,
                                            unsigned char* lds, int dxmode = 0, int mask = 0) {
  const int nch = LOWER ? D.nch_fs : D.nch_bs;
  const int* ptr = LOWER ? m.fs_ptr : m.bs_ptr;
  const int* blob = LOWER ? m.fs_blob : m.bs_blob;
  ChunkStager<!RES> stg(ptr, blob, nch, lds, tid, nt);
  for (int ch = 0; ch < nch; ++ch) {
    const int* h = stg.get(ch);
    const int nrow = h[0];
    const int4* rw = reinterpret_cast<const int4*>(h + 4);
    const int* cols = reinterpret_cast<const int*>(rw + nrow + 1);
    const Grp g = groups(nrow, tid, nt, gmin);
    const int G = g.G;
    const int s = g.lane % S, e = g.lane / S, E = G / S;
    for (int ri = g.gid; ri < nrow; ri += g.ng) {
      const int4 r = rw[ri];   // row, first position, -, first column
      const int a = r.x, n = rw[ri + 1].w - r.w;
      // the row's own right-hand side (and, backward, its pivot inverse and
      // the correction it adds to) are loaded before the dot product, so
      // that their latency overlaps it
      T ya0 = T(0), ya1 = T(0);
      Blk<T> Di = {T(0), T(0), T(0), T(0)};
      double dx0 = 0.0, dx1 = 0.0;
      if (e == 0) {
        ya0 = c.y[sP<S>(a, s)];
        ya1 = c.y[sP<S>(a, s) + 1];
        if (!LOWER) Di = ld_blk(c.dinv + sB<S>(a, s));
        if (!LOWER && dxmode == 2) {
          dx0 = c.dx[sP<S>(a, s)];
          dx1 = c.dx[sP<S>(a, s) + 1];
        }
      }
      T s0 = T(0), s1 = T(0);
      int j = e;
      // HBM-resident slices: two entries per round, loads first, summed in
      // order (in LDS the loads return quickly and the plain loop is shorter)
      for (; !RES && j + E < n; j += 2 * E) {
        Blk<T> M[2];
        T z[2][2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int p = r.y + j + u * E;
          M[u] = ld_blk_nt(c.lu + sB<S>(p, s));
          const int k = cols[r.w + j + u * E];
          z[u][0] = c.y[sP<S>(k, s)];
          z[u][1] = c.y[sP<S>(k, s) + 1];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          s0 += M[u].a * z[u][0] + M[u].b * z[u][1];
          s1 += M[u].c * z[u][0] + M[u].d * z[u][1];
        }
      }
      for (; j < n; j += E) {
        const Blk<T> M = RES ? ld_blk(c.lu + sB<S>(r.y + j, s)) : ld_blk_nt(c.lu + sB<S>(r.y + j, s));
        const int k = cols[r.w + j];
        const T z0 = c.y[sP<S>(k, s)], z1 = c.y[sP<S>(k, s) + 1];
        s0 += M.a * z0 + M.b * z1;
        s1 += M.c * z0 + M.d * z1;
      }
      s0 = group_sum<T, S>(s0, G);
      s1 = group_sum<T, S>(s1, G);
      if (e == 0) {
        if (LOWER) {
          c.y[sP<S>(a, s)] = ya0 - s0;
          c.y[sP<S>(a, s) + 1] = ya1 - s1;
        } else {
          const T t0 = ya0 - s0, t1 = ya1 - s1;
          const T x0 = Di.a * t0 + Di.b * t1, x1 = Di.c * t0 + Di.d * t1;
          c.y[sP<S>(a, s)] = x0;
          c.y[sP<S>(a, s) + 1] = x1;
          if (dxmode == 1) {
            c.dx[sP<S>(a, s)] = double(x0);
            c.dx[sP<S>(a, s) + 1] = double(x1);
          } else if (dxmode == 2 && ((mask >> s) & 1)) {
            c.dx[sP<S>(a, s)] = dx0 + double(x0);
            c.dx[sP<S>(a, s) + 1] = dx1 + double(x1);
          }
        }
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// dense tail: the top rows of the elimination tree, one wavefront per
// scenario, with no workgroup barrier inside

__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// ----------------------------------------------------------------------------
// the tail of HBM-resident slices in an LDS copy: its tail-column blocks in a
// compact numbering (tl), its pivot inverses (td) and right-hand sides (ty),
// each scenario's copy contiguous so that the lanes of the wavefront that
// works on it read different banks.  The blocks are copied in after the
// barrier-synchronised part of the factorisation, factored and solved there
// one wavefront per scenario, and written back only when the factors are
// kept.  The tail program (records of every pivot row: its pivot block,
// masks of its blocks left and right of the diagonal, the rows below it)
// stays in LDS (tq) for the whole launch; the factorisation's update words
// are staged in the metadata area or read in place (tp).

__device__ __forceinline__ int tcB(int cb, int s, int nbs) { return (s * nbs + cb) * 4; }
__device__ __forceinline__ int tdB(int k, int s, int t) { return (s * t + k) * 4; }
__device__ __forceinline__ int tyP(int k, int s, int t) { return (s * t + k) * 2; }

template <typename T, int S>
__device__ __forceinline__ void ltail_copy(const Sym& m, const Dims& D, St<T>& c, T* tl, int tid, int nt,
                                           bool out) {
  const int nq = D.tail_nblk * S * 4;
  for (int q = tid; q < nq; q += nt) {
    const int comp = q & 3, s = (q >> 2) % S, cb = (q >> 2) / S;
    T* g = c.lu + sB<S>(m.tail_cblk[cb], s) + comp;
    T* x = tl + tcB(cb, s, D.tail_nbs) + comp;
    if (out) *g = *x;
    else *x = *g;
  }
}

template <typename T, int S>
__device__ __forceinline__ void ltail_store_dinv(const Dims& D, St<T>& c, const T* td, int tid, int nt) {
  for (int q = tid; q < D.tail_t * S * 4; q += nt) {
    const int comp = q & 3, s = (q >> 2) % S, k = (q >> 2) / S;
    c.dinv[sB<S>(D.tail_base + k, s) + comp] = td[tdB(k, s, D.tail_t) + comp];
  }
}

template <typename T, int S>
__device__ __forceinline__ void ltail_load_dinv(const Dims& D, St<T>& c, T* td, int tid, int nt) {
  for (int q = tid; q < D.tail_t * S * 4; q += nt) {
    const int comp = q & 3, s = (q >> 2) % S, k = (q >> 2) / S;
    td[tdB(k, s, D.tail_t) + comp] = c.dinv[sB<S>(D.tail_base + k, s) + comp];
  }
}

// ty: the tail rows' right-hand sides for the fused forward solve, written
// back at the end.  Every lane inverts the pivot block itself from its LDS
// copy (a broadcast read); the updates of one pivot have distinct targets
// outside its row and column, so the lanes take them two at a time with
// every load issued first; the rows' multipliers L(i, k) D_k^-1 replace
// their blocks only after all updates have read them.
template <typename T, int S>
__device__ __forceinline__ void ltail_factor(const Dims& D, St<T>& c, T* tl, T* td, T* ty, const int* tq,
                                             const int* tp, int tid, int nt, bool fwd, int* piv) {
  const int t = D.tail_t, tb = D.tail_base, nbs = D.tail_nbs;
  const int w = tid >> 6, l = tid & 63, nw = nt >> 6;
  for (int s = w; s < S; s += nw) {
    if (fwd && l < t) {
      ty[tyP(l, s, t)] = c.y[sP<S>(tb + l, s)];
      ty[tyP(l, s, t) + 1] = c.y[sP<S>(tb + l, s) + 1];
    }
    asm volatile("" ::: "memory");
    for (int k = 0; k < t; ++k) {
      const int4 r = reinterpret_cast<const int4*>(tq)[2 * k];   // pivot, first U, nu | ns << 16, steps
      const int uoff = tq[8 * k + 4];
      const Blk<T> Dk = ld_blk(tl + tcB(r.x, s, nbs));
      const T det = Dk.a * Dk.d - Dk.b * Dk.c;
      const T inv = recip(det);
      const Blk<T> Di = {Dk.d * inv, -Dk.b * inv, -Dk.c * inv, Dk.a * inv};
      if (l == 0) {
        // pivots of the block: a, then the Schur complement d - c b / a
        const T eps = sizeof(T) == 8 ? T(1e-14) : T(1e-7);
        const bool zero = !(fabs(Dk.a) > eps * (fabs(Dk.a) + fabs(Dk.b))) ||
                          !(fabs(det) > eps * fabs(Dk.a) * (fabs(Dk.c) + fabs(Dk.d))) ||
                          !isfinite(inv);
        if (zero) piv[s] = 1;
        st_blk(td + tdB(k, s, t), Di);
      }
      const int nu = r.z & 0xffff, ns = r.z >> 16;
      const unsigned* up = reinterpret_cast<const unsigned*>(tp + (uoff - D.tail_prog_prefix));
      const int np = nu * ns;
      for (int q = l; q < np; q += 128) {
        const bool two = q + 64 < np;
        const unsigned r0 = up[q], r1 = two ? up[q + 64] : r0;
        T* a0 = tl + tcB((int)(r0 & 2047u), s, nbs);
        T* a1 = tl + tcB((int)(r1 & 2047u), s, nbs);
        const Blk<T> L0 = ld_blk(tl + tcB((int)((r0 >> 11) & 2047u), s, nbs));
        const Blk<T> U0 = ld_blk(tl + tcB(r.y + (int)(r0 >> 22), s, nbs));
        const Blk<T> L1 = ld_blk(tl + tcB((int)((r1 >> 11) & 2047u), s, nbs));
        const Blk<T> U1 = ld_blk(tl + tcB(r.y + (int)(r1 >> 22), s, nbs));
        Blk<T> x0 = ld_blk(a0), x1 = ld_blk(a1);
        const Blk<T> M0 = mul(mul(L0, Di), U0), M1 = mul(mul(L1, Di), U1);
        x0.a -= M0.a; x0.b -= M0.b; x0.c -= M0.c; x0.d -= M0.d;
        x1.a -= M1.a; x1.b -= M1.b; x1.c -= M1.c; x1.d -= M1.d;
        st_blk(a0, x0);
        if (two) st_blk(a1, x1);
      }
      asm volatile("" ::: "memory");
      if (l < ns) {
        const int sw = tq[r.w + l], lc = sw & 0xffff, ir = sw >> 16;
        const Blk<T> L = mul(ld_blk(tl + tcB(lc, s, nbs)), Di);
        st_blk(tl + tcB(lc, s, nbs), L);
        if (fwd) {
          const T yk0 = ty[tyP(k, s, t)], yk1 = ty[tyP(k, s, t) + 1];
          ty[tyP(ir, s, t)] -= L.a * yk0 + L.b * yk1;
          ty[tyP(ir, s, t) + 1] -= L.c * yk0 + L.d * yk1;
        }
      }
      // the next pivot reads what this one wrote: LDS operations of a
      // wavefront complete in order, so only the compiler must keep it
      asm volatile("" ::: "memory");
    }
    if (fwd && l < t) {
      c.y[sP<S>(tb + l, s)] = ty[tyP(l, s, t)];
      c.y[sP<S>(tb + l, s) + 1] = ty[tyP(l, s, t) + 1];
    }
  }
}

// stages the tail program's update words into the metadata area (when they
// fit there); returns where the factorisation reads them
__device__ __forceinline__ const int* ltail_updates(const Sym& m, const Dims& D, unsigned char* stg, int tid,
                                                    int nt) {
  const int* src = m.tail_prog + D.tail_prog_prefix;
  if (!D.tail_prog_lds) return src;
  int* dst = reinterpret_cast<int*>(stg);
  for (int q = tid; q < D.tail_prog_ints - D.tail_prog_prefix; q += nt) dst[q] = src[q];
  return dst;
}

// the triangular solves of the tail: lane l < t holds the right-hand side
// of tail row l in registers, solved values reach the other lanes by lane
// broadcast, and each lane walks its own row's blocks (consecutive compact
// indices located by the row's masks) with the next two loaded ahead of use

// forward solve of scenario s's tail rows (lanes l and l + 32 share row l
// for the terms on rows outside the tail: their L blocks left of the tail,
// against unknowns already solved, four in flight per lane, the two partial
// sums meeting by a lane swap); the result stays in y0, y1
template <typename T, int S>
__device__ __forceinline__ void ltail_fs_one(const Sym& m, const Dims& D, St<T>& c, const T* tl, const int* tq,
                                             int s, int l, T& y0, T& y1, const T* pa = nullptr, int P = 0) {
  const int t = D.tail_t, tb = D.tail_base, nbs = D.tail_nbs;
  const int lr = l & 31, hs = l >> 5;
  T o0 = T(0), o1 = T(0);
  y0 = T(0);
  y1 = T(0);
  if (pa) {
    // the terms were summed by the whole workgroup: P parts per row, added
    // in part order by lane l (lanes l + 32 add nothing)
    if (l < t) {
      y0 = c.y[sP<S>(tb + l, s)];
      y1 = c.y[sP<S>(tb + l, s) + 1];
      for (int h = 0; h < P; ++h) {
        o0 += pa[((s * t + l) * P + h) * 2];
        o1 += pa[((s * t + l) * P + h) * 2 + 1];
      }
    }
  } else if (lr < t) {
    const int a = tb + lr;
    if (hs == 0) {
      y0 = c.y[sP<S>(a, s)];
      y1 = c.y[sP<S>(a, s) + 1];
    }
    const int p1 = m.tail_split[lr];
    for (int p = m.rp[a] + hs; p < p1; p += 8) {
      Blk<T> L[4];
      T z[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int pu = p + 2 * u;
        const bool in = pu < p1;
        const int k = in ? m.ci[pu] : 0;
        L[u] = in ? ld_blk(c.lu + sB<S>(pu, s)) : Blk<T>{T(0), T(0), T(0), T(0)};
        z[u][0] = c.y[sP<S>(k, s)];
        z[u][1] = c.y[sP<S>(k, s) + 1];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        o0 += L[u].a * z[u][0] + L[u].b * z[u][1];
        o1 += L[u].c * z[u][0] + L[u].d * z[u][1];
      }
    }
  }
  if (!pa) {
    o0 += __shfl_xor(o0, 32);
    o1 += __shfl_xor(o1, 32);
  }
  y0 -= o0;
  y1 -= o1;
  unsigned mk = l < t ? (unsigned)tq[8 * l + 5] : 0u;
  int idx = l < t ? tq[8 * l] - __popc(mk) : 0;   // the row's first block left of the diagonal
  const Blk<T> Z = {T(0), T(0), T(0), T(0)};
  Blk<T> L0 = mk ? ld_blk(tl + tcB(idx, s, nbs)) : Z;
  Blk<T> L1 = (mk & (mk - 1)) ? ld_blk(tl + tcB(idx + 1, s, nbs)) : Z;
  for (int k = 0; k + 1 < t; ++k) {
    const T yk0 = lane_bcast(y0, k), yk1 = lane_bcast(y1, k);
    if (mk & (1u << k)) {   // k is the lowest column left to do
      y0 -= L0.a * yk0 + L0.b * yk1;
      y1 -= L0.c * yk0 + L0.d * yk1;
      mk &= mk - 1;
      ++idx;
      L0 = L1;
      if (mk & (mk - 1)) L1 = ld_blk(tl + tcB(idx + 1, s, nbs));
    }
  }
}

// backward solve of scenario s's tail rows, right-hand sides in y0, y1
template <typename T, int S>
__device__ __forceinline__ void ltail_bs_one(const Dims& D, const T* tl, const T* td, const int* tq, int s,
                                             int l, T& y0, T& y1) {
  const int t = D.tail_t, nbs = D.tail_nbs;
  const Blk<T> Z = {T(0), T(0), T(0), T(0)};
  Blk<T> Di = Z;
  unsigned mk = 0u;
  int idx = 0;
  if (l < t) {
    Di = ld_blk(td + tdB(l, s, t));
    mk = (unsigned)tq[8 * l + 6];
    idx = tq[8 * l] + __popc(mk);   // the row's last block right of the diagonal
  }
  Blk<T> U0 = mk ? ld_blk(tl + tcB(idx, s, nbs)) : Z;
  Blk<T> U1 = (mk & (mk - 1)) ? ld_blk(tl + tcB(idx - 1, s, nbs)) : Z;
  for (int j = t - 1; j >= 0; --j) {
    if (l == j) {
      const T x0 = Di.a * y0 + Di.b * y1, x1 = Di.c * y0 + Di.d * y1;
      y0 = x0;
      y1 = x1;
    }
    if (j == 0) break;
    const T xj0 = lane_bcast(y0, j), xj1 = lane_bcast(y1, j);
    if (mk & (1u << j)) {   // j is the highest column left to do
      y0 -= U0.a * xj0 + U0.b * xj1;
      y1 -= U0.c * xj0 + U0.d * xj1;
      mk &= ~(1u << j);
      --idx;
      U0 = U1;
      if (mk & (mk - 1)) U1 = ld_blk(tl + tcB(idx - 1, s, nbs));
    }
  }
}

// writes the solved tail rows: y, and dx = y (dxmode 1) or dx += y (dxmode
// 2, scenarios in mask; dx loaded by the caller ahead of the solve)
template <typename T, int S>
__device__ __forceinline__ void ltail_put(const Dims& D, St<T>& c, int s, int l, T y0, T y1, int dxmode, int mask,
                                          double dx0, double dx1) {
  if (l >= D.tail_t) return;
  const int a = D.tail_base + l;
  c.y[sP<S>(a, s)] = y0;
  c.y[sP<S>(a, s) + 1] = y1;
  if (dxmode == 1) {
    c.dx[sP<S>(a, s)] = double(y0);
    c.dx[sP<S>(a, s) + 1] = double(y1);
  } else if (dxmode == 2 && ((mask >> s) & 1)) {
    c.dx[sP<S>(a, s)] = dx0 + double(y0);
    c.dx[sP<S>(a, s) + 1] = dx1 + double(y1);
  }
}

template <typename T, int S>
__device__ __forceinline__ void ltail_dx(const Dims& D, St<T>& c, int s, int l, int dxmode, double& dx0,
                                         double& dx1) {
  dx0 = dx1 = 0.0;
  if (dxmode == 2 && l < D.tail_t) {
    dx0 = c.dx[sP<S>(D.tail_base + l, s)];
    dx1 = c.dx[sP<S>(D.tail_base + l, s) + 1];
  }
}

// backward solve after the factorisation (its forward solve was fused in)
template <typename T, int S>
__device__ __forceinline__ void ltail_bsolve(const Dims& D, St<T>& c, const T* tl, const T* td, const int* tq,
                                             int tid, int nt, int dxmode = 0, int mask = 0) {
  const int w = tid >> 6, l = tid & 63, nw = nt >> 6;
  for (int s = w; s < S; s += nw) {
    T y0 = T(0), y1 = T(0);
    double dx0, dx1;
    ltail_dx<T, S>(D, c, s, l, dxmode, dx0, dx1);
    if (l < D.tail_t) {
      y0 = c.y[sP<S>(D.tail_base + l, s)];
      y1 = c.y[sP<S>(D.tail_base + l, s) + 1];
    }
    ltail_bs_one<T, S>(D, tl, td, tq, s, l, y0, y1);
    ltail_put<T, S>(D, c, s, l, y0, y1, dxmode, mask, dx0, dx1);
  }
}

// forward then backward solve of the tail rows (refinement), the forward
// result kept in registers.  The terms of the tail rows on rows outside the
// tail are summed by the whole workgroup first: thread (row l, part h,
// scenario s), scenarios fastest, so that the lanes of a wavefront read the
// slice's interleaved blocks and unknowns in contiguous runs, adds entries
// h, h + P, ... of row l (four in flight), and its sum lands in LDS (pa, the
// metadata area, free here); the row's lane adds the parts in order
template <typename T, int S>
__device__ __forceinline__ void ltail_fbsolve(const Sym& m, const Dims& D, St<T>& c, const T* tl, const T* td,
                                              const int* tq, int tid, int nt, int dxmode, int mask,
                                              unsigned char* stg) {
  const int w = tid >> 6, l = tid & 63, nw = nt >> 6;
  const int t = D.tail_t;
  T* pa = nullptr;
  int P = 0;
  if (t > 0) {
    P = nt / (S * t);
    const int cap = (int)((4 * (size_t)D.chunk_ints) / (2 * sizeof(T) * S * t));
    P = P < cap ? P : cap;
    P = P < 32 ? P : 32;
    if (P >= 1) {
      pa = reinterpret_cast<T*>(stg);
      for (int q = tid; q < S * t * P; q += nt) {
        const int s = q % S, h = (q / S) % P, lr = q / (S * P);
        const int a = D.tail_base + lr;
        const int p1 = m.tail_split[lr];
        T o0 = T(0), o1 = T(0);
        for (int p = m.rp[a] + h; p < p1; p += 4 * P) {
          Blk<T> L[4];
          T z[4][2];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int pu = p + u * P;
            const bool in = pu < p1;
            const int k = in ? m.ci[pu] : 0;
            L[u] = in ? ld_blk(c.lu + sB<S>(pu, s)) : Blk<T>{T(0), T(0), T(0), T(0)};
            z[u][0] = c.y[sP<S>(k, s)];
            z[u][1] = c.y[sP<S>(k, s) + 1];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            o0 += L[u].a * z[u][0] + L[u].b * z[u][1];
            o1 += L[u].c * z[u][0] + L[u].d * z[u][1];
          }
        }
        pa[((s * t + lr) * P + h) * 2] = o0;
        pa[((s * t + lr) * P + h) * 2 + 1] = o1;
      }
      __syncthreads();
    }
  }
  for (int s = w; s < S; s += nw) {
    T y0, y1;
    double dx0, dx1;
    ltail_dx<T, S>(D, c, s, l, dxmode, dx0, dx1);
    ltail_fs_one<T, S>(m, D, c, tl, tq, s, l, y0, y1, pa, P);
    ltail_bs_one<T, S>(D, tl, td, tq, s, l, y0, y1);
    ltail_put<T, S>(D, c, s, l, y0, y1, dxmode, mask, dx0, dx1);
  }
}

// ----------------------------------------------------------------------------
// register-resident dense tail (LDS-resident slices): wavefront w handles the
// tail of scenario w.  Lanes 2l and 2l + 1 hold the two scalar rows of tail
// block row l (components a b, resp. c d, of every 2x2 block), as register
// vectors: L part left of the diagonal, the inverted pivot block on it, U
// part right of it.  The column loops are unrolled over the register
// capacity, so each column is a fixed register and a structurally zero block
// costs one uniform branch (per-pivot structure masks); only the pivot
// column is indexed at run time (register-indexing mode, no scratch).  Pivot
// blocks, U rows and solved unknowns reach the other lanes by lane broadcast.
// Same arithmetic, in the same order, as the sparse per-pivot elimination.

// tail block row of a lane (lanes 2l and 2l + 1), made opaque to the
// compiler at each use: otherwise the per-column lane masks of the unrolled
// loops (l == j, l < j for every j) are hoisted out of the Newton loop and
// live in spilled scalar registers, which costs more to reload than to
// recompute
__device__ __forceinline__ int lane_row(int ln) {
  int l = ln >> 1;
  asm volatile("" : "+v"(l));
  return l;
}

// register capacity of the dense tail, in block rows (one 32-dword register
// tuple per scalar-row half)
template <typename T>
constexpr int tail_cap() { return sizeof(T) == 4 ? 32 : 16; }

template <typename T>
struct TailRow {
  typedef T V __attribute__((ext_vector_type(tail_cap<T>())));
  V p, q;   // this lane's scalar row of block j: (p[j], q[j])
};

// the partner lane's value (lanes 2l <-> 2l + 1) by a DPP quad permutation
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// this lane's scalar row of the tail blocks (l, j), j < t, into R.  Every
// register-vector index in the tail code below is a compile-time constant
// (unrolled column loops with uniform skips), except the pivot column of the
// factorisation.
template <typename T, int S>
__device__ __forceinline__ void rt_load(const Sym& m, const Dims& D, const St<T>& c, int s, int l, int h,
                                        TailRow<T>& R) {
  R = TailRow<T>{};
  const int t = __builtin_amdgcn_readfirstlane(D.tail_t);
  constexpr int C = tail_cap<T>();
  // eight columns at a time, their index and value loads issued together
#pragma unroll
  for (int jb = 0; jb < C; jb += 8) {
    if (jb >= t) break;
    int p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = jb + u;
      p[u] = (j < t && l < t) ? m.tail_pos[l * t + j] : -1;
    }
    T x0[8], x1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x0[u] = T(0);
      x1[u] = T(0);
      if (p[u] >= 0) {
        const T* b = c.lu + sB<S>(p[u], s) + 2 * h;
        x0[u] = b[0];
        x1[u] = b[1];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) { R.p[jb + u] = x0[u]; R.q[jb + u] = x1[u]; }
  }
}

// LU of the tail rows pivot by pivot, kept in R for the tail solves of the
// iteration; with fwd, the forward solve of the tail rows' right-hand sides
// is fused in
template <typename T, int S>
__device__ __forceinline__ void rt_factor(const Sym& m, const Dims& D, St<T>& c, int s, int ln, bool fwd,
                                          int* piv, TailRow<T>& R) {
  const int t = __builtin_amdgcn_readfirstlane(D.tail_t), tb = D.tail_base;
  if (t == 0) return;
  const int l = lane_row(ln), h = ln & 1;
  rt_load<T, S>(m, D, c, s, l, h, R);
  T y = T(0);   // component h of the right-hand side of row l
  if (fwd && l < t) y = c.y[sP<S>(tb + l, s) + h];
  // this lane's row of its own pivot block as it was when eliminated, for
  // the pivot test after the loop
  T pvp = T(0), pvq = T(0);
  // the structure mask of the next pivot is loaded one pivot ahead, so its
  // LDS latency hides behind the current pivot's work
  unsigned mnext = m.tail_mask[0];
  for (int k = 0; k < t; ++k) {
    const unsigned mk = __builtin_amdgcn_readfirstlane(mnext);   // U columns j > k
    if (k + 1 < t) mnext = m.tail_mask[k + 1];
    const T xp = R.p[k], xq = R.q[k];
    const T da = lane_bcast(xp, 2 * k), db = lane_bcast(xq, 2 * k);
    const T dc = lane_bcast(xp, 2 * k + 1), dd = lane_bcast(xq, 2 * k + 1);
    const T det = da * dd - db * dc;
    const T inv = recip(det);
    const T ia = dd * inv, ib = -db * inv, ic = -dc * inv, id = da * inv;
    pvp = l == k ? xp : pvp;
    pvq = l == k ? xq : pvq;
    const bool below = l > k && l < t;
    // row h of A_lk D_k^-1 on the rows below the pivot, zero elsewhere, so
    // that the update below needs no per-lane select; every lane forms the
    // products and selects by value (no divergent branch around the
    // register-indexed writes)
    const T m0 = xp * ia + xq * ic, m1 = xp * ib + xq * id;
    const T l0 = below ? m0 : T(0), l1 = below ? m1 : T(0);
    const T np = below ? m0 : (l == k ? (h ? ic : ia) : xp);
    const T nq = below ? m1 : (l == k ? (h ? id : ib) : xq);
    R.p[k] = np;
    R.q[k] = nq;
    if (fwd) {
      const T yk0 = lane_bcast(y, 2 * k), yk1 = lane_bcast(y, 2 * k + 1);
      y -= l0 * yk0 + l1 * yk1;
    }
    // eight columns per uniform test, then one test per column
#pragma unroll
    for (int jb = 0; jb < tail_cap<T>(); jb += 8) {
      if ((mk >> jb) & 0xFFu) {
#pragma unroll
        for (int j = jb; j < jb + 8; ++j) {
          if ((mk >> j) & 1u) {
            const T ua = lane_bcast(R.p[j], 2 * k), ub = lane_bcast(R.q[j], 2 * k);
            const T uc = lane_bcast(R.p[j], 2 * k + 1), ud = lane_bcast(R.q[j], 2 * k + 1);
            R.p[j] -= l0 * ua + l1 * uc;
            R.q[j] -= l0 * ub + l1 * ud;
          }
        }
      }
    }
  }
  // the pivot test of every block at once (the same arithmetic as at its
  // elimination): a, then the Schur complement d - c b / a, must stand out
  // of the block's scale, and the inverse must be finite
  {
    const T op = pair_swap(pvp), oq = pair_swap(pvq);
    const T da = h ? op : pvp, db = h ? oq : pvq, dc = h ? pvp : op, dd = h ? pvq : oq;
    const T det = da * dd - db * dc;
    const T inv = recip(det);
    const T eps = sizeof(T) == 8 ? T(1e-14) : T(1e-7);
    const bool zero = l < t && (!(fabs(da) > eps * (fabs(da) + fabs(db))) ||
                                !(fabs(det) > eps * fabs(da) * (fabs(dc) + fabs(dd))) || !isfinite(inv));
    if (__ballot(zero) && ln == 0) piv[s] = 1;
  }
  if (fwd && l < t) c.y[sP<S>(tb + l, s) + h] = y;
}

// the tail factors back into the slice's storage (multipliers and U blocks
// in place, inverted pivots to dinv), for the adjoint
template <typename T, int S>
__device__ __forceinline__ void rt_store(const Sym& m, const Dims& D, St<T>& c, int s, int ln,
                                         const TailRow<T>& R) {
  const int t = __builtin_amdgcn_readfirstlane(D.tail_t), tb = D.tail_base;
  const int l = lane_row(ln), h = ln & 1;
  constexpr int C = tail_cap<T>();
#pragma unroll
  for (int jb = 0; jb < C; jb += 8) {
    if (jb >= t) break;
    int p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = jb + u;
      p[u] = -1;
      if (j < t && l < t) p[u] = j == l ? -2 : m.tail_pos[l * t + j];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const T xp = R.p[jb + u], xq = R.q[jb + u];
      T* b = nullptr;
      if (p[u] == -2) b = c.dinv + sB<S>(tb + l, s) + 2 * h;
      else if (p[u] >= 0) b = c.lu + sB<S>(p[u], s) + 2 * h;
      if (b) { b[0] = xp; b[1] = xq; }
    }
  }
}

// forward solve of the tail rows: their terms on rows outside the tail,
// then the unit block-lower tail block
template <typename T, int S>
__device__ __forceinline__ void rt_fsolve(const Sym& m, const Dims& D, St<T>& c, int s, int ln,
                                          const TailRow<T>& R) {
  const int t = __builtin_amdgcn_readfirstlane(D.tail_t), tb = D.tail_base;
  if (t == 0) return;
  const int l = lane_row(ln), h = ln & 1;
  T y = T(0);
  if (l < t) {
    const int a = tb + l;
    y = c.y[sP<S>(a, s) + h];
    for (int p = m.rp[a]; p < m.tail_split[l]; ++p) {
      const T* b = c.lu + sB<S>(p, s) + 2 * h;
      const int k = m.ci[p];
      y -= b[0] * c.y[sP<S>(k, s)] + b[1] * c.y[sP<S>(k, s) + 1];
    }
  }
  const unsigned lm = __builtin_amdgcn_readfirstlane(m.tail_mask[t]);   // columns with L blocks
#pragma unroll
  for (int j = 0; j < tail_cap<T>(); ++j) {
    if ((lm >> j) & 1u) {
      const T yj0 = lane_bcast(y, 2 * j), yj1 = lane_bcast(y, 2 * j + 1);
      if (l > j && l < t) y -= R.p[j] * yj0 + R.q[j] * yj1;
    }
  }
  if (l < t) c.y[sP<S>(tb + l, s) + h] = y;
}

// backward solve of the tail block, the last unknown first
template <typename T, int S>
__device__ __forceinline__ void rt_bsolve(const Sym& m, const Dims& D, St<T>& c, int s, int ln,
                                          const TailRow<T>& R, int dxmode = 0, int mask = 0) {
  const int t = __builtin_amdgcn_readfirstlane(D.tail_t), tb = D.tail_base;
  if (t == 0) return;
  const int l = lane_row(ln), h = ln & 1;
  T y = T(0);
  double dxo = 0.0;
  if (l < t) {
    y = c.y[sP<S>(tb + l, s) + h];
    if (dxmode == 2) dxo = c.dx[sP<S>(tb + l, s) + h];
  }
  const unsigned cm = __builtin_amdgcn_readfirstlane(m.tail_mask[t + 1]);   // columns with U blocks
#pragma unroll
  for (int j = tail_cap<T>() - 1; j >= 0; --j) {
    if (j < t) {
      const T xp = R.p[j], xq = R.q[j];
      // x_j = D_j^-1 y_j on the two lanes of row j: row h of the inverse
      // times both components (the partner lane holds the other one)
      const T yo = pair_swap(y);
      if (l == j) y = xp * (h ? yo : y) + xq * (h ? y : yo);
      if ((cm >> j) & 1u) {
        const T xj0 = lane_bcast(y, 2 * j), xj1 = lane_bcast(y, 2 * j + 1);
        if (l < j) y -= xp * xj0 + xq * xj1;
      }
    }
  }
  if (l < t) {
    c.y[sP<S>(tb + l, s) + h] = y;
    if (dxmode == 1) c.dx[sP<S>(tb + l, s) + h] = double(y);
    else if (dxmode == 2 && ((mask >> s) & 1)) c.dx[sP<S>(tb + l, s) + h] = dxo + double(y);
  }
}

// dV = V (d|V|/|V| + j dtheta) for the correction dx (slack: 0); four items
// per thread, loads first
// (with the state in HBM, 1/|V| is formed from e and f: one stream fewer)
template <typename T, int S, bool RES>
__device__ __forceinline__ void phase_dv(const Sym& m, const Dims& D, St<T>& c, int tid, int nt) {
  // HBM: four items in flight per thread; LDS-resident slices hold fewer
  // items than threads, and the spare items' loads only cost LDS issue slots
  constexpr int U = RES ? 1 : 4;
  const int s = tid % S, N = D.n_bus * S;
  for (int base = tid; base < N; base += U * nt) {
    double dth[U], dvm[U], rv[U], e[U], f[U];
    int a[U], bt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * nt;
      const int o = idx < N ? idx : base;
      a[u] = m.bus_blk[o / S];
      bt[u] = m.bus_type[o / S];
      const int pa = a[u] >= 0 ? a[u] : 0;
      const int go = c.g(o / S, s);
      dth[u] = c.dx[sP<S>(pa, s)];
      dvm[u] = c.dx[sP<S>(pa, s) + 1];
      rv[u] = RES ? c.rvm[go] : 0.0;
      e[u] = c.e[go];
      f[u] = c.f[go];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + u * nt;
      if (idx >= N) continue;
      double dvr = 0.0, dvi = 0.0;
      if (a[u] >= 0) {
        if (!RES) rv[u] = rsqrt_nr(e[u] * e[u] + f[u] * f[u]);
        const double rho = bt[u] == 0 ? dvm[u] * rv[u] : 0.0;
        dvr = e[u] * rho - f[u] * dth[u];
        dvi = f[u] * rho + e[u] * dth[u];
      }
      const int go = c.g(idx / S, s);
      c.dvr[go] = dvr;
      c.dvi[go] = dvi;
    }
  }
  __syncthreads();
}

// r = -F1 - J1 dx in FP64 without forming J1: J1 dx = -(dS restricted to the
// F1 rows), dS = dV conj(I) + V conj(Y dV).  Result cast into y; with norm,
// ||r||_inf per scenario lands in the scratch maxima.
template <typename T, int S>
__device__ __forceinline__ void phase_residual(const Sym& m, const Dims& D, St<T>& c, int tid, int nt,
                                               bool norm, unsigned char* scr) {
  double mx = 0.0;
  const int s = tid % S, N = D.n_bus * S;
  for (int base = tid; base < N; base += kBusU * nt) {
    int i[kBusU], a[kBusU], bt[kBusU];
    bool v[kBusU];
    double e[kBusU], f[kBusU], ir[kBusU], ii[kBusU], dvr[kBusU], dvi[kBusU], F0[kBusU], F1[kBusU];
#pragma unroll
    for (int u = 0; u < kBusU; ++u) {
      const int idx = base + u * nt;
      const int o = idx < N ? idx : base;
      i[u] = o / S;
      a[u] = m.bus_blk[i[u]];
      bt[u] = m.bus_type[i[u]];
      v[u] = idx < N && a[u] >= 0;
      const int go = c.g(i[u], s);
      e[u] = c.e[go];
      f[u] = c.f[go];
      ir[u] = c.ire[go];
      ii[u] = c.iim[go];
      dvr[u] = c.dvr[go];
      dvi[u] = c.dvi[go];
      const int pa = a[u] >= 0 ? a[u] : 0;
      F0[u] = c.F[sP<S>(i[u], s)];
      F1[u] = c.F[sP<S>(i[u], s) + 1];
    }
    double dir[kBusU], dii[kBusU];
    yrow_multi<S, kBusU, kBusW>(m, c.dvr, c.dvi, c.gs, i, s, v, dir, dii);
#pragma unroll
    for (int u = 0; u < kBusU; ++u) {
      if (!v[u]) continue;
      const double dSr = dvr[u] * ir[u] + dvi[u] * ii[u] + e[u] * dir[u] + f[u] * dii[u];
      const double dSi = dvi[u] * ir[u] - dvr[u] * ii[u] + f[u] * dir[u] - e[u] * dii[u];
      const int o = sP<S>(a[u], s);
      const double r0 = -F0[u] + dSr;
      const double r1 = bt[u] == 0 ? -F1[u] + dSi : 0.0;
      c.y[o] = T(r0);
      c.y[o + 1] = T(r1);
      mx = fmax(mx, fmax(fabs(r0), fabs(r1)));
    }
  }
  __syncthreads();
  if (norm) block_max<S>(mx, 0, scr, tid, nt);
}

// loss gradients on the Step-2 outputs as extra weights of the transposed
// product through Y_bus: dL/dp_g on the slack row (dP), dL/dq_g on PV and
// slack rows (dQ).  These rows are exactly the ones outside F1, so they never
// collide with the lambda weights.  [batch][n_bus] arrays, either may be null.
struct GenW {
  const double *p = nullptr, *q = nullptr;
  int b0 = 0, count = 0, n = 0;
  __device__ __forceinline__ bool on() const { return p || q; }
  __device__ __forceinline__ void add(int i, int s, int bt, double& nr, double& ni) const {
    const int b = b0 + s;
    if (b >= count) return;
    const size_t o = (size_t)b * n + i;
    if (p && bt == 2) nr += p[o];
    if (q && bt != 0) ni += q[o];
  }
};

// e + jf from (|V|, theta) for the scenarios in `mask`
// (1/|V| is stored only for LDS-resident slices: the passes over HBM state
// form it from e and f)
template <typename T, int S, bool RES>
__device__ __forceinline__ void phase_set_state(const Dims& D, St<T>& c, int tid, int nt, int mask) {
  for (int idx = tid; idx < D.n_bus * S; idx += nt) {
    if (!((mask >> (idx % S)) & 1)) continue;
    const int o = c.g(idx / S, idx % S);
    double sn, cs;
    sincos(c.va[idx], &sn, &cs);
    const double v = c.vm[o];
    c.e[o] = v * cs;
    c.f[o] = v * sn;
    if (RES) c.rvm[o] = 1.0 / v;
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------
// the Newton kernel: one workgroup = one slice of S scenarios

template <typename T, bool RES, int S>
__global__ void __launch_bounds__(RES ? res_newton_threads<T>() : 1024) k_newton(KParams kp) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, nt = blockDim.x;
  PhaseClock pc(tid);
  const int slice = blockIdx.x;
  const Dims& D = kp.dims;
  unsigned char* scr = smem;
  int* piv = reinterpret_cast<int*>(scr + kPivOff);
  const double* fnr = reinterpret_cast<const double*>(scr + kFnOff);
  const int* bdr = reinterpret_cast<const int*>(scr + kBadOff);
  int* s_it = reinterpret_cast<int*>(scr + kItOff);
  int* s_st = reinterpret_cast<int*>(scr + kStOff);
  double* s_fn = reinterpret_cast<double*>(scr + kFnvOff);

  const unsigned char* mbase = kp.sym;
  if (RES) {   // the shared symbolic image, once per workgroup, 16 bytes per lane
    int4* dst = reinterpret_cast<int4*>(smem + kScratchBytes);
    const int4* src = reinterpret_cast<const int4*>(kp.sym);
    for (int q = tid; q < (kp.so.newton_bytes >> 4); q += nt) dst[q] = src[q];
    mbase = smem + kScratchBytes;
  }
  const Sym m = bind_sym(mbase, kp.sym, kp.so);
  St<T> c;
  if (RES) {
    double* d = reinterpret_cast<double*>(smem + kScratchBytes + kp.so.newton_bytes);
    c = bind_state<T, S>(d, reinterpret_cast<T*>(d + (size_t)kp.llay.sd * S), kp.llay);
  } else {
    c = bind_state<T, S>(kp.wsl_d + (size_t)slice * S * kp.lay.sd,
                         reinterpret_cast<T*>(kp.wsl_t) + (size_t)slice * S * kp.lay.st, kp.lay);
  }
  if (tid < S) { piv[tid] = 0; s_it[tid] = 0; s_st[tid] = 0; s_fn[tid] = 0.0; }
  pc.count(PH_NEWTON_LAUNCHES);

  const int n = D.n_bus, nb = D.nb;
  int act = 0;   // scenarios of the slice still iterating (identical in every thread)
  for (int s = 0; s < S; ++s)
    if (slice * S + s < kp.count) act |= 1 << s;

  // inputs: specified injections and the start point; padding scenarios of
  // the last slice get an empty problem and are never written back
  for (int idx = tid; idx < n * S; idx += nt) {
    const int i = idx / S, s = idx % S;
    const int b = slice * S + s;
    const int bt = m.bus_type[i];
    if (b < kp.count) {
      const size_t o = (size_t)b * n + i;
      const double pg = (kp.pg && bt == 1) ? kp.pg[o] : 0.0;
      c.ps[idx] = pg - kp.pd[o];
      c.qs[idx] = -kp.qd[o];
      if (kp.mode == MODE_SOLVE) {
        c.vm[c.g(i, s)] = bt == 0 ? 1.0 : kp.vset[o];
        c.va[idx] = 0.0;
      } else {
        c.vm[c.g(i, s)] = kp.vm_in[o];
        c.va[idx] = bt == 2 ? 0.0 : kp.va_in[o];
      }
    } else {
      c.ps[idx] = 0.0;
      c.qs[idx] = 0.0;
      c.vm[c.g(i, s)] = 1.0;
      c.va[idx] = 0.0;
    }
  }
  __syncthreads();
  phase_set_state<T, S, RES>(D, c, tid, nt, (1 << S) - 1);

  const bool mixed = sizeof(T) == 4;
  const int gmin = kp.gmin > S ? kp.gmin : S;
  const int wv = tid >> 6, ln = tid & 63;   // LDS-resident tails: wavefront wv <-> scenario wv
  unsigned char* stg = smem + kScratchBytes; // HBM-resident slices: staged level metadata
  T* tl = reinterpret_cast<T*>(smem + kScratchBytes + 4 * (size_t)kp.dims.chunk_ints);   // HBM: LDS tail
  T* td = tl + (size_t)kp.dims.tail_nbs * S * 4;
  T* ty = td + (size_t)kp.dims.tail_t * S * 4;
  int* tq = reinterpret_cast<int*>(ty + (size_t)kp.dims.tail_t * S * 2);   // HBM: tail program prefix
  if constexpr (!RES) {
    for (int q = tid; q < kp.dims.tail_prog_prefix; q += nt) tq[q] = m.tail_prog[q];
    // the right-hand side / solution of the triangular solves, when the
    // slice's copy fits in LDS: every solve's gathers then stay on chip
    if (kp.dims.y_lds_off) c.y = reinterpret_cast<T*>(smem + kp.dims.y_lds_off);
  }
  TailRow<T> R;                             // this wavefront's factored tail rows
  // slices of several scenarios hand the backward solves' results to dx as
  // they write them
  constexpr bool fuse = S > 1 && !RES;
  constexpr int dx_set = fuse ? 1 : 0, dx_add = fuse ? 2 : 0;
  pc.mark(PH_SETUP);
  while (true) {
    if constexpr (RES && sizeof(T) == 8) phase_mismatch_lds<T, S>(m, D, c, tid, nt, scr);
    else phase_mismatch<T, S>(m, D, c, tid, nt, scr);
    pc.mark(PH_MISMATCH);
    for (int s = 0; s < S; ++s) {
      if (!((act >> s) & 1)) continue;
      const double f = fnr[s];
      int st = -1;
      if (bdr[s]) st = 2;
      else if (kp.mode == MODE_SOLVE && f < kp.tol) st = 0;
      else if (kp.mode == MODE_SOLVE && s_it[s] >= kp.max_iter) st = 1;
      if (tid == 0) s_fn[s] = f;
      if (st >= 0) {
        act &= ~(1 << s);
        if (tid == 0) s_st[s] = st;
      }
    }
    if (kp.mode == MODE_EVAL_MISMATCH || kp.mode == MODE_EVAL_FACTOR) break;
    if (kp.mode == MODE_EVAL_FILL) {
      phase_fill<T, S, RES>(m, D, c, tid, nt);
      break;
    }
    if (!act) break;
    // slices of several scenarios hand the backward solves' results to dx
    // as they write them; a slice of one scenario scatters each of those
    // stores to its own line, on the critical path of a level, so it updates
    // dx in a streaming pass of its own
    phase_fill<T, S, RES>(m, D, c, tid, nt);
    pc.mark(PH_FILL);
    pc.count(PH_NEWTON_STEPS);
    phase_factor<T, S, RES>(m, D, c, tid, nt, gmin, true, piv, stg);
    pc.mark(PH_FACTOR_LEVELS);
    if constexpr (RES) {
      if (wv < S) rt_factor<T, S>(m, D, c, wv, ln, true, piv, R);
    } else {
      ltail_copy<T, S>(m, D, c, tl, tid, nt, false);
      const int* tp = ltail_updates(m, D, stg, tid, nt);
      __syncthreads();
      ltail_factor<T, S>(D, c, tl, td, ty, tq, tp, tid, nt, true, piv);
    }
    __syncthreads();
    pc.mark(PH_FACTOR_TAIL);
    for (int s = 0; s < S; ++s)
      if (((act >> s) & 1) && piv[s]) {
        act &= ~(1 << s);
        if (tid == 0) s_st[s] = 3;
      }
    if (!act) break;
    if constexpr (RES) {
      if (wv < S) rt_bsolve<T, S>(m, D, c, wv, ln, R, dx_set);
    } else {
      ltail_bsolve<T, S>(D, c, tl, td, tq, tid, nt, dx_set);
    }
    __syncthreads();
    pc.mark(PH_BSOLVE_TAIL);
    phase_solve<T, S, RES, false>(m, D, c, tid, nt, gmin, stg, dx_set);   // dx = y as well
    pc.mark(PH_BSOLVE_LEVELS);
    // slices that keep dx out of the backward solves hand the last solve's
    // y to dx only when a later pass reads dx: the state update reads dx
    // (pend 0), y (pend 1: dx = y) or dx + y (pend 2, scenarios in pmask)
    int pend = fuse ? 0 : 1, pmask = 0;
    auto settle = [&]() {
      if (pend == 1) {
        for (int q = tid; q < 2 * nb * S; q += nt) c.dx[q] = double(c.y[q]);
        __syncthreads();
      } else if (pend == 2) {
        for (int q = tid; q < 2 * nb * S; q += nt)
          if ((pmask >> ((q >> 1) % S)) & 1) c.dx[q] += double(c.y[q]);
        __syncthreads();
      }
      pend = 0;
    };
    if (mixed) {
      int ref = act;   // scenarios still refining their correction
      for (int r = 0; r < kp.refine; ++r) {
        pc.mark(PH_OTHER);
        settle();
        phase_dv<T, S, RES>(m, D, c, tid, nt);
        pc.mark(PH_REFINE_DV);
        phase_residual<T, S>(m, D, c, tid, nt, kp.adaptive, scr);
        pc.mark(PH_REFINE_RESIDUAL);
        if (kp.adaptive) {
          // inexact-Newton forcing term: refine while the FP64 residual of the
          // correction exceeds max(min(0.1, |F|) |F|, 0.1 tol)
          for (int s = 0; s < S; ++s) {
            const double f = s_fn[s];
            const double thr = fmax(fmin(0.1, f) * f, 0.1 * kp.tol);
            if (!(fnr[s] > thr)) ref &= ~(1 << s);
          }
          if (!ref) break;
        }
        pc.count(PH_REFINE_STEPS);
        phase_solve<T, S, RES, true>(m, D, c, tid, nt, gmin, stg);
        pc.mark(PH_REFINE_FSOLVE_LEVELS);
        if constexpr (RES) {
          if (wv < S) {
            rt_fsolve<T, S>(m, D, c, wv, ln, R);
            rt_bsolve<T, S>(m, D, c, wv, ln, R, dx_add, ref);
          }
        } else {
          ltail_fbsolve<T, S>(m, D, c, tl, td, tq, tid, nt, dx_add, ref, stg);
        }
        __syncthreads();
        pc.mark(PH_REFINE_TAIL);
        phase_solve<T, S, RES, false>(m, D, c, tid, nt, gmin, stg, dx_add, ref);   // dx += y as well
        pc.mark(PH_REFINE_BSOLVE_LEVELS);
        if (!fuse) {
          pend = 2;
          pmask = ref;
        }
      }
    }
    if (kp.mode == MODE_EVAL_STEP) {
      settle();
      break;
    }
    // state update of the active scenarios (theta on non-slack buses, |V| on
    // PQ buses) and their e + jf, by the thread that owns the item in both
    for (int idx = tid; idx < n * S; idx += nt) {
      const int i = idx / S, s = idx % S;
      if (!((act >> s) & 1)) continue;
      const int a = m.bus_blk[i], o = c.g(i, s);
      double va = c.va[idx], vm = c.vm[o];
      if (a >= 0) {
        const int p = sP<S>(a, s);
        const bool with_y = pend == 1 || (pend == 2 && ((pmask >> s) & 1));
        const double d0 = (pend == 1 ? 0.0 : c.dx[p]) + (with_y ? double(c.y[p]) : 0.0);
        const double d1 = (pend == 1 ? 0.0 : c.dx[p + 1]) + (with_y ? double(c.y[p + 1]) : 0.0);
        va += d0;
        if (m.bus_type[i] == 0) vm += d1;
        c.va[idx] = va;
        c.vm[o] = vm;
      }
      double sn, cs;
      if (RES) {
        sincos(va, &sn, &cs);
      } else {
        const double2 r = sincos_call(va);
        sn = r.x;
        cs = r.y;
      }
      c.e[o] = vm * cs;
      c.f[o] = vm * sn;
      if (RES) c.rvm[o] = 1.0 / vm;
    }
    __syncthreads();
    if (tid < S && ((act >> tid) & 1)) s_it[tid]++;
    pc.mark(PH_OTHER);
  }
  __syncthreads();
  pc.mark(PH_OTHER);

  // outputs
  if (kp.mode == MODE_SOLVE) {
    for (int idx = tid; idx < n * S; idx += nt) {
      const int i = idx / S, s = idx % S;
      const int b = slice * S + s;
      if (b < kp.count) {
        kp.vm_out[(size_t)b * n + i] = c.vm[c.g(i, s)];
        kp.va_out[(size_t)b * n + i] = c.va[idx];
      }
    }
    if (tid < S && slice * S + tid < kp.count) {
      const int b = slice * S + tid;
      if (kp.iters_out) kp.iters_out[b] = s_it[tid];
      if (kp.status_out) kp.status_out[b] = s_st[tid];
      if (kp.fnorm_out) kp.fnorm_out[b] = s_st[tid] == 2 ? __builtin_nan("") : s_fn[tid];
    }
  } else if (kp.mode == MODE_EVAL_FILL) {
    // the filled LU values of each scenario, block by block (row-major 2x2)
    const size_t nv = 4 * (size_t)D.nnzb;
    for (int q = tid; q < 4 * D.nnzb * S; q += nt) {
      const int blk = q >> 2, b = slice * S + blk % S;
      if (b < kp.count) kp.out[(size_t)b * nv + 4 * (blk / S) + (q & 3)] = double(c.lu[q]);
    }
  } else if (kp.mode == MODE_EVAL_MISMATCH || kp.mode == MODE_EVAL_STEP) {
    const int nj = D.nj;
    for (int idx = tid; idx < n * S; idx += nt) {
      const int i = idx / S, s = idx % S;
      const int b = slice * S + s;
      const int a = m.bus_blk[i];
      if (b >= kp.count || a < 0) continue;
      double* o = kp.out + (size_t)b * nj;
      if (kp.mode == MODE_EVAL_MISMATCH) {
        o[m.ord_p[i]] = c.F[sP<S>(i, s)];
        if (m.bus_type[i] == 0) o[D.npvpq + m.ord_q[i]] = c.F[sP<S>(i, s) + 1];
      } else {
        o[D.npq + m.ord_p[i]] = c.dx[sP<S>(a, s)];
        if (m.bus_type[i] == 0) o[m.ord_q[i]] = c.dx[sP<S>(a, s) + 1];
      }
    }
  }
  // keep the converged state and the factors of J1 at it for the adjoint
  const bool keep = (kp.mode == MODE_SOLVE && kp.keep) || kp.mode == MODE_EVAL_FACTOR;
  if (keep) {
    if (tid < S) piv[tid] = 0;
    phase_fill<T, S, RES>(m, D, c, tid, nt);
    phase_factor<T, S, RES>(m, D, c, tid, nt, gmin, false, piv, stg);
    if constexpr (RES) {
      if (wv < S) {
        rt_factor<T, S>(m, D, c, wv, ln, false, piv, R);
        rt_store<T, S>(m, D, c, wv, ln, R);
      }
    } else {
      ltail_copy<T, S>(m, D, c, tl, tid, nt, false);
      const int* tp = ltail_updates(m, D, stg, tid, nt);
      __syncthreads();
      ltail_factor<T, S>(D, c, tl, td, ty, tq, tp, tid, nt, false, piv);
      __syncthreads();
      ltail_copy<T, S>(m, D, c, tl, tid, nt, true);
      ltail_store_dinv<T, S>(D, c, td, tid, nt);
    }
    __syncthreads();
    if (tid < S && s_st[tid] == 0 && piv[tid]) s_st[tid] = 3;
    pc.mark(PH_KEEP);
    // LDS-resident slices: the kept state and factors go to the per-scenario
    // workspace, which the adjoint copies into its own LDS slices; the
    // HBM-resident adjoint reads this slice workspace in place
    if (RES) {
      for (int s = 0; s < S; ++s) {
        const int b = slice * S + s;
        if (b >= kp.count) break;
        double* gd = kp.ws_d + (size_t)b * kp.lay.sd;
        T* gt = reinterpret_cast<T*>(kp.ws_t) + (size_t)b * kp.lay.st;
        for (int q = tid; q < 4 * D.nnzb; q += nt) gt[kp.lay.o_lu + q] = c.lu[sB<S>(q >> 2, s) + (q & 3)];
        for (int q = tid; q < 4 * nb; q += nt) gt[kp.lay.o_dinv + q] = c.dinv[sB<S>(q >> 2, s) + (q & 3)];
        for (int i = tid; i < n; i += nt) {
          const int gi = i * kp.lay.gk;   // the per-scenario workspace groups them
          gd[kp.lay.o_e + gi] = c.e[c.g(i, s)];
          gd[kp.lay.o_f + gi] = c.f[c.g(i, s)];
          gd[kp.lay.o_vm + gi] = c.vm[c.g(i, s)];
          gd[kp.lay.o_va + i] = c.va[sI<S>(i, s)];
        }
      }
    }
    __syncthreads();
  }
  if (tid < S && slice * S + tid < kp.count) {
    int* gi = kp.ws_i + (size_t)(slice * S + tid) * 4;
    gi[0] = keep ? s_st[tid] : -1;
    gi[1] = s_it[tid];
  }
  pc.mark(PH_OUTPUT);
}

// direct Step-2 terms of the gradients: z2 carries the load of its own row
// with unit weight (p_g,R = P_R + p_d,R, q_g = Q + q_d on PV and slack
// buses), and the completed p_g on PV buses is x's p_g passed through
__device__ __forceinline__ void gen_direct(const KParams& kp, size_t o, int bt, double& gpd, double& gqd,
                                           double& gpg) {
  if (kp.mode != MODE_SOLVE) return;
  // value selects, so that the three sums stay in registers
  const double gp = kp.g_pgo ? kp.g_pgo[o] : 0.0;
  const double gq = (kp.g_qgo && bt != 0) ? kp.g_qgo[o] : 0.0;
  gpd = (kp.g_pgo && bt == 2) ? gpd + gp : gpd;
  gpg = (kp.g_pgo && bt == 1) ? gpg + gp : gpg;
  gqd = (kp.g_qgo && bt != 0) ? gqd + gq : gqd;
}

// ----------------------------------------------------------------------------
// adjoint slices: S scenarios per workgroup.  LDS-resident (small grids):
// the kept state and factors copied into LDS, level metadata chunks in place
// in the LDS image.  HBM-resident: the slice workspace of the forward solve
// (state and factors interleaved by scenario) read in place, metadata chunks
// staged in LDS.  The transposed dense tail in registers, one wavefront per
// scenario.  U^T then L^T with the kept factors (transposed blocks read
// through the mirror-position map), FP64-residual refinement for FP32
// factors, then the gradient assembly with J3^T lambda (and vbar2) as one
// transposed product through Y_bus.

// metadata of the transposed solves
struct AdjSym {
  const int *ut_ptr, *ut_blob, *lt_ptr, *lt_blob, *tt_ptr, *tt_pairs;
};

__device__ __forceinline__ AdjSym bind_adj(const unsigned char* b, const SymOffsets& o) {
  auto I = [](const unsigned char* x, int off) { return reinterpret_cast<const int*>(x + off); };
  return {I(b, o.ut_ptr), I(b, o.ut_blob), I(b, o.lt_ptr), I(b, o.lt_blob), I(b, o.tt_ptr), I(b, o.tt_pairs)};
}

// U^T w = g by forward levels (UT) or L^T l = w by backward levels, rows
// outside the tail, in place in y; entries are (column, position of the
// transposed block) pairs
template <typename T, int S, bool RES, bool UT>
__device__ __forceinline__ void phase_tsolve(const AdjSym& a, const Dims& D, St<T>& c, int tid, int nt, int gmin,
                                             unsigned char* lds) {
  const int nch = UT ? D.nch_ut : D.nch_lt;
  const int* ptr = UT ? a.ut_ptr : a.lt_ptr;
  const int* blob = UT ? a.ut_blob : a.lt_blob;
  ChunkStager<!RES> stg(ptr, blob, nch, lds, tid, nt);
  for (int ch = 0; ch < nch; ++ch) {
    const int* h = stg.get(ch);
    const int nrow = h[0];
    const int4* rw = reinterpret_cast<const int4*>(h + 4);
    const int* cols = reinterpret_cast<const int*>(rw + nrow + 1);
    const Grp g = groups(nrow, tid, nt, gmin);
    const int G = g.G;
    const int s = g.lane % S, e = g.lane / S, E = G / S;
    for (int ri = g.gid; ri < nrow; ri += g.ng) {
      const int4 r = rw[ri];   // row, -, -, first pair
      const int row = r.x, n = rw[ri + 1].w - r.w;
      // the row's own right-hand side (and, for U^T, its pivot inverse)
      // loaded before the dot product, whose latency they then overlap
      T ya0 = T(0), ya1 = T(0);
      Blk<T> Di = {T(0), T(0), T(0), T(0)};
      if (e == 0) {
        ya0 = c.y[sP<S>(row, s)];
        ya1 = c.y[sP<S>(row, s) + 1];
        if (UT) Di = ld_blk(c.dinv + sB<S>(row, s));
      }
      T s0 = T(0), s1 = T(0);
      int j = e;
      for (; !RES && j + E < n; j += 2 * E) {   // HBM: two entries per round, loads first, in order
        Blk<T> B[2];
        T z[2][2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int k = cols[2 * (r.w + j + u * E)], mp = cols[2 * (r.w + j + u * E) + 1];
          B[u] = ld_blk(c.lu + sB<S>(mp, s));
          z[u][0] = c.y[sP<S>(k, s)];
          z[u][1] = c.y[sP<S>(k, s) + 1];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          s0 += B[u].a * z[u][0] + B[u].c * z[u][1];
          s1 += B[u].b * z[u][0] + B[u].d * z[u][1];
        }
      }
      for (; j < n; j += E) {
        const int k = cols[2 * (r.w + j)], mp = cols[2 * (r.w + j) + 1];
        const Blk<T> B = ld_blk(c.lu + sB<S>(mp, s));
        const T z0 = c.y[sP<S>(k, s)], z1 = c.y[sP<S>(k, s) + 1];
        s0 += B.a * z0 + B.c * z1;
        s1 += B.b * z0 + B.d * z1;
      }
      s0 = group_sum<T, S>(s0, G);
      s1 = group_sum<T, S>(s1, G);
      if (e == 0) {
        if (UT) {
          const T t0 = ya0 - s0, t1 = ya1 - s1;
          c.y[sP<S>(row, s)] = Di.a * t0 + Di.c * t1;
          c.y[sP<S>(row, s) + 1] = Di.b * t0 + Di.d * t1;
        } else {
          c.y[sP<S>(row, s)] = ya0 - s0;
          c.y[sP<S>(row, s) + 1] = ya1 - s1;
        }
      }
    }
    __syncthreads();
  }
}

// transposed solves of the tail rows, one wavefront per scenario, lanes 2l
// and 2l + 1 = the two scalar rows of tail row l: lane row h of block j is
// column h of the stored block (j, l) (U_jl^T left of the diagonal, the
// transposed inverted pivot on it, L_jl^T right of it).  U^T forward (after
// the terms on rows outside the tail), then L^T backward.
// With tl (HBM-resident slices) the tail blocks come from the LDS tail copy
// (tl, td, located through the tail program's records tq) instead of the
// slice workspace, and the terms on rows outside the tail from the parts pa
// (P per row) the whole workgroup summed beforehand.
template <typename T, int S>
__device__ __forceinline__ void rt_tsolve(const Sym& m, const AdjSym& a, const Dims& D, St<T>& c, int s, int ln,
                                          const T* tl = nullptr, const T* td = nullptr, const int* tq = nullptr,
                                          const T* pa = nullptr, int P = 0) {
  const int t = __builtin_amdgcn_readfirstlane(D.tail_t), tb = D.tail_base;
  if (t == 0) return;
  const int l = lane_row(ln), h = ln & 1;
  TailRow<T> R = TailRow<T>{};
  constexpr int C = tail_cap<T>();
#pragma unroll
  for (int jb = 0; jb < C; jb += 8) {
    if (jb >= t) break;
    int p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = jb + u;
      p[u] = -1;
      if (j < t && l < t) {
        if (j == l) {
          p[u] = -2;
        } else if (tl) {
          // compact index of block (j, l): row j's blocks are consecutive
          // in column order, located by its masks
          const int dk = tq[8 * j];
          const unsigned lm = (unsigned)tq[8 * j + 5], um = (unsigned)tq[8 * j + 6];
          const unsigned below = (1u << l) - 1u;
          if (j < l && ((um >> l) & 1u)) p[u] = dk + 1 + __popc(um & below);
          else if (j > l && ((lm >> l) & 1u)) p[u] = dk - __popc(lm) + __popc(lm & below);
        } else {
          p[u] = m.tail_pos[j * t + l];
        }
      }
    }
    T x0[8], x1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x0[u] = T(0);
      x1[u] = T(0);
      const T* b = nullptr;
      if (tl) b = p[u] == -2 ? td + tdB(l, s, t) : (p[u] >= 0 ? tl + tcB(p[u], s, D.tail_nbs) : nullptr);
      else b = p[u] == -2 ? c.dinv + sB<S>(tb + l, s) : (p[u] >= 0 ? c.lu + sB<S>(p[u], s) : nullptr);
      if (b) { x0[u] = b[h]; x1[u] = b[2 + h]; }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) { R.p[jb + u] = x0[u]; R.q[jb + u] = x1[u]; }
  }
  T y = T(0);
  if (l < t && pa) {
    y = c.y[sP<S>(tb + l, s) + h];
    T acc = T(0);
    for (int hp = 0; hp < P; ++hp) acc += pa[((s * t + l) * P + hp) * 2 + h];
    y -= acc;
  } else if (l < t) {
    const int row = tb + l;
    y = c.y[sP<S>(row, s) + h];
    // the terms on rows outside the tail, four pairs in flight
    const int q1 = a.tt_ptr[l + 1];
    T acc = T(0);
    for (int q = a.tt_ptr[l]; q < q1; q += 4) {
      T b0[4], b1[4], z0[4], z1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool in = q + u < q1;
        const int k = in ? a.tt_pairs[2 * (q + u)] : 0, mp = in ? a.tt_pairs[2 * (q + u) + 1] : 0;
        const T* b = c.lu + sB<S>(mp, s);
        b0[u] = in ? b[h] : T(0);
        b1[u] = in ? b[2 + h] : T(0);
        z0[u] = c.y[sP<S>(k, s)];
        z1[u] = c.y[sP<S>(k, s) + 1];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += b0[u] * z0[u] + b1[u] * z1[u];
    }
    y -= acc;
  }
  const unsigned lm = __builtin_amdgcn_readfirstlane(m.tail_mask[t]);
  const unsigned cm = __builtin_amdgcn_readfirstlane(m.tail_mask[t + 1]);
#pragma unroll
  for (int j = 0; j < C; ++j) {   // U^T w = g
    if (j < t) {
      const T xp = R.p[j], xq = R.q[j];
      const T yo = pair_swap(y);
      if (l == j) y = xp * (h ? yo : y) + xq * (h ? y : yo);
      if ((lm >> j) & 1u) {
        const T w0 = lane_bcast(y, 2 * j), w1 = lane_bcast(y, 2 * j + 1);
        if (l > j && l < t) y -= xp * w0 + xq * w1;
      }
    }
  }
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {   // L^T lambda = w
    if ((cm >> j) & 1u) {
      const T z0 = lane_bcast(y, 2 * j), z1 = lane_bcast(y, 2 * j + 1);
      if (l < j) y -= R.p[j] * z0 + R.q[j] * z1;
    }
  }
  if (l < t) c.y[sP<S>(tb + l, s) + h] = y;
}

// HBM-resident adjoint slices: the terms of the tail rows of U^T on rows
// outside the tail, summed by the whole workgroup before the tail solves
// (thread (row l, part h, scenario s), scenarios fastest, adds pairs h,
// h + P, ... of row l, four in flight) into LDS parts (lds, the metadata
// area, free between the two transposed solves); returns the parts, P per
// row, or nullptr when not even one part per row fits
template <typename T, int S>
__device__ __forceinline__ const T* tt_parts(const AdjSym& a, const Dims& D, St<T>& c, int tid, int nt,
                                             unsigned char* lds, int& P) {
  const int t = D.tail_t;
  P = 0;
  if (t == 0) return nullptr;
  P = nt / (S * t);
  const int cap = (int)((4 * (size_t)D.chunk_ints) / (2 * sizeof(T) * S * t));
  P = P < cap ? P : cap;
  P = P < 32 ? P : 32;
  if (P < 1) return nullptr;
  T* pa = reinterpret_cast<T*>(lds);
  for (int q = tid; q < S * t * P; q += nt) {
    const int s = q % S, h = (q / S) % P, lr = q / (S * P);
    const int q1 = a.tt_ptr[lr + 1];
    T o0 = T(0), o1 = T(0);
    for (int p = a.tt_ptr[lr] + h; p < q1; p += 4 * P) {
      Blk<T> B[4];
      T z[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int pu = p + u * P;
        const bool in = pu < q1;
        const int k = in ? a.tt_pairs[2 * pu] : 0, mp = in ? a.tt_pairs[2 * pu + 1] : 0;
        B[u] = in ? ld_blk(c.lu + sB<S>(mp, s)) : Blk<T>{T(0), T(0), T(0), T(0)};
        z[u][0] = c.y[sP<S>(k, s)];
        z[u][1] = c.y[sP<S>(k, s) + 1];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        o0 += B[u].a * z[u][0] + B[u].c * z[u][1];
        o1 += B[u].b * z[u][0] + B[u].d * z[u][1];
      }
    }
    pa[((s * t + lr) * P + h) * 2] = o0;
    pa[((s * t + lr) * P + h) * 2 + 1] = o1;
  }
  __syncthreads();
  return pa;
}

// adjoint residual r = g - J1^T lam in FP64 without forming J1 (transposed
// directional derivative of S = V conj(Y V)), on an interleaved slice: with
// nu = lam_P + j lam_Q (plus the Step-2 weights) and
// c_m = conj(nu_m I_m) + sum_i Y_im nu_i conj(V_i),
//   (J1^T lam)_theta_m = Im(V_m c_m),  (J1^T lam)_|V|m = -Re(V_m c_m) / |V_m|.
// Also stores Re(V_m c_m) / |V_m| = -(J3^T lam)_m for every bus in aux.
// g == nullptr: only aux; to_y: r into y (factor precision); otherwise r
// replaces g in place.
template <typename T, int S>
__device__ __forceinline__ void phase_adj_residual_s(const Sym& m, const Dims& D, St<T>& c, int tid, int nt,
                                                     const double* lam, double* g, bool to_y,
                                                     GenW gw = GenW{}) {
  for (int idx = tid; idx < D.n_bus * S; idx += nt) {   // w_i = nu_i conj(V_i)
    const int i = idx / S, s = idx % S, o = c.g(i, s);
    const int a = m.bus_blk[i];
    double nr = 0.0, ni = 0.0;
    if (a >= 0 && lam) { nr = lam[sP<S>(a, s)]; ni = m.bus_type[i] == 0 ? lam[sP<S>(a, s) + 1] : 0.0; }
    gw.add(i, s, m.bus_type[i], nr, ni);
    const double e = c.e[o], f = c.f[o];
    c.dvr[o] = nr * e + ni * f;
    c.dvi[o] = ni * e - nr * f;
  }
  __syncthreads();
  for (int idx = tid; idx < D.n_bus * S; idx += nt) {
    const int mb = idx / S, s = idx % S, o = c.g(mb, s);
    // sum over the row's entries of Y_im w_i, four entries per round with
    // their loads issued together, in column order
    double tr = 0.0, ti = 0.0;
    const int q1 = m.y_rp[mb + 1];
    for (int q = m.y_rp[mb]; q < q1; q += 4) {
      int j[4];
      double yg[4], yb[4], wr[4], wi[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const bool in = q + w < q1;
        j[w] = in ? m.y_ci[q + w] : 0;
        const int qt = in ? m.y_tr[q + w] : 0;   // position of Y_im
        yg[w] = in ? m.y_g[qt] : 0.0;
        yb[w] = in ? m.y_b[qt] : 0.0;
      }
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        wr[w] = c.dvr[c.g(j[w], s)];
        wi[w] = c.dvi[c.g(j[w], s)];
      }
#pragma unroll
      for (int w = 0; w < 4; ++w)
        if (q + w < q1) {
          tr += yg[w] * wr[w] - yb[w] * wi[w];
          ti += yg[w] * wi[w] + yb[w] * wr[w];
        }
    }
    const int a = m.bus_blk[mb];
    double nr = 0.0, ni = 0.0;
    if (a >= 0 && lam) { nr = lam[sP<S>(a, s)]; ni = m.bus_type[mb] == 0 ? lam[sP<S>(a, s) + 1] : 0.0; }
    gw.add(mb, s, m.bus_type[mb], nr, ni);
    const double ir = c.ire[o], ii = c.iim[o];
    const double cr = (nr * ir - ni * ii) + tr;      // Re c_m
    const double ci = -(nr * ii + ni * ir) + ti;     // Im c_m
    const double e = c.e[o], f = c.f[o], vm = c.vm[o];
    const double vcr = e * cr - f * ci;               // Re(V_m c_m)
    const double vci = e * ci + f * cr;               // Im(V_m c_m)
    c.aux[idx] = vcr / vm;
    if (a >= 0 && g) {
      const double r0 = g[sP<S>(a, s)] - vci;
      const double r1 = m.bus_type[mb] == 0 ? g[sP<S>(a, s) + 1] + vcr / vm : 0.0;
      if (to_y) { c.y[sP<S>(a, s)] = T(r0); c.y[sP<S>(a, s) + 1] = T(r1); }
      else { g[sP<S>(a, s)] = r0; g[sP<S>(a, s) + 1] = r1; }   // in place
    }
  }
  __syncthreads();
}

template <typename T, bool RES, int S>
__global__ void __launch_bounds__(RES ? kResThreads : 1024) k_adjoint_slice(KParams kp) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int slice = blockIdx.x;
  const Dims& D = kp.dims;
  int* s_ok = reinterpret_cast<int*>(smem + kPivOff);
  unsigned char* stg = smem + kScratchBytes;   // HBM: staged metadata chunks
  const unsigned char* img = RES ? smem + kScratchBytes : kp.sym;
  if (RES) {   // the shared image prefix (Newton arrays, then the adjoint's), 16 bytes per lane
    int4* dst = reinterpret_cast<int4*>(smem + kScratchBytes);
    const int4* src = reinterpret_cast<const int4*>(kp.sym);
    for (int q = tid; q < (kp.so.adj_bytes >> 4); q += nt) dst[q] = src[q];
  }
  Sym m = bind_sym(img, kp.sym, kp.so);
  m.y_tr = reinterpret_cast<const int*>(img + kp.so.y_tr);
  const AdjSym as = bind_adj(img, kp.so);
  St<T> c;
  if (RES) {
    double* dbase = reinterpret_cast<double*>(smem + kScratchBytes + kp.so.adj_bytes);
    c = bind_state<T, S>(dbase, reinterpret_cast<T*>(dbase + (size_t)kp.alay.sd * S), kp.alay);
  } else {
    c = bind_state<T, S>(kp.wsl_d + (size_t)slice * S * kp.lay.sd,
                         reinterpret_cast<T*>(kp.wsl_t) + (size_t)slice * S * kp.lay.st, kp.lay);
    // the solve vector in LDS where the Newton kernel keeps it there too (the
    // workgroup has the same LDS)
    if (kp.dims.y_lds_off) c.y = reinterpret_cast<T*>(smem + kp.dims.y_lds_off);
  }
  const int n = D.n_bus, nb = D.nb;
  const bool eval = kp.mode == MODE_EVAL_ADJOINT;
  const int wv = tid >> 6, ln = tid & 63, nw = nt >> 6;

  // kept state and factors of the slice's scenarios (padding scenarios: flat, identity)
  if (RES) {
  for (int idx = tid; idx < n * S; idx += nt) {
    const int i = idx / S, s = idx % S;
    const int b = slice * S + s;
    double e = 1.0, f = 0.0, v = 1.0;
    if (b < kp.count) {
      const double* gd = kp.ws_d + (size_t)b * kp.lay.sd;
      const int gi = i * kp.lay.gk;
      e = gd[kp.lay.o_e + gi];
      f = gd[kp.lay.o_f + gi];
      v = gd[kp.lay.o_vm + gi];
    }
    c.e[c.g(i, s)] = e;
    c.f[c.g(i, s)] = f;
    c.vm[c.g(i, s)] = v;
  }
  for (int q = tid; q < 4 * D.nnzb * S; q += nt) {
    const int comp = q & 3, blk = q >> 2, p = blk / S, s = blk % S;
    const int b = slice * S + s;
    c.lu[q] = b < kp.count ? reinterpret_cast<const T*>(kp.ws_t)[(size_t)b * kp.lay.st + kp.lay.o_lu + 4 * p + comp]
                           : T(0);
  }
  for (int q = tid; q < 4 * nb * S; q += nt) {
    const int comp = q & 3, blk = q >> 2, p = blk / S, s = blk % S;
    const int b = slice * S + s;
    c.dinv[q] = b < kp.count ? reinterpret_cast<const T*>(kp.ws_t)[(size_t)b * kp.lay.st + kp.lay.o_dinv + 4 * p + comp]
                             : ((comp == 0 || comp == 3) ? T(1) : T(0));
  }
  }
  // HBM-resident slices: the factored tail in LDS, as the Newton kernel
  // lays it out (the same LDS size), with the tail program's records
  T* tl = nullptr;
  T* td = nullptr;
  int* tq = nullptr;
  if constexpr (!RES) {
    tl = reinterpret_cast<T*>(smem + kScratchBytes + 4 * (size_t)D.chunk_ints);
    td = tl + (size_t)D.tail_nbs * S * 4;
    tq = reinterpret_cast<int*>(td + (size_t)D.tail_t * S * 4 + (size_t)D.tail_t * S * 2);
    for (int q = tid; q < D.tail_prog_prefix; q += nt) tq[q] = m.tail_prog[q];
    ltail_copy<T, S>(m, D, c, tl, tid, nt, false);
    ltail_load_dinv<T, S>(D, c, td, tid, nt);
  }
  if (tid < S) {
    const int b = slice * S + tid;
    s_ok[tid] = b < kp.count && kp.ws_i[(size_t)b * 4] == 0;
  }
  __syncthreads();
  // I at the kept state (HBM-resident slices: the forward kernel's last
  // mismatch left it in the slice workspace, at the same state), g_z1 per
  // block into F
  for (int idx = tid; idx < n * S; idx += nt) {
    const int i = idx / S, s = idx % S;
    const int b = slice * S + s;
    if (RES) {
      double ir[1], ii[1];
      const int ib[1] = {i};
      const bool vb[1] = {true};
      yrow_multi<S, 1, 4>(m, c.e, c.f, c.gs, ib, s, vb, ir, ii);
      c.ire[c.g(i, s)] = ir[0];
      c.iim[c.g(i, s)] = ii[0];
    }
    const int a = m.bus_blk[i];
    if (a < 0) continue;
    double g0 = 0.0, g1 = 0.0;
    if (b < kp.count) {
      if (eval) {
        const double* rhs = kp.rhs + (size_t)b * D.nj;
        g0 = rhs[D.npq + m.ord_p[i]];
        g1 = m.bus_type[i] == 0 ? rhs[m.ord_q[i]] : 0.0;
      } else {
        g0 = kp.g_va[(size_t)b * n + i];
        g1 = m.bus_type[i] == 0 ? kp.g_vm[(size_t)b * n + i] : 0.0;
      }
    }
    c.F[sP<S>(a, s)] = g0;
    c.F[sP<S>(a, s) + 1] = g1;
  }
  __syncthreads();
  // Step 2: g_z1 += vbar2 on z1 (vbar2 = -J2^T dL/dz2, a transposed product)
  GenW gw;
  if (!eval) { gw.p = kp.g_pgo; gw.q = kp.g_qgo; gw.b0 = slice * S; gw.count = kp.count; gw.n = n; }
  if (gw.on()) phase_adj_residual_s<T, S>(m, D, c, tid, nt, nullptr, c.F, false, gw);
  for (int q = tid; q < 2 * nb * S; q += nt) c.y[q] = T(c.F[q]);
  __syncthreads();
  const int gmin = S > 4 ? S : 4;
  auto solve = [&]() {
    phase_tsolve<T, S, RES, true>(as, D, c, tid, nt, gmin, stg);
    if constexpr (RES) {
      for (int s = wv; s < S; s += nw) rt_tsolve<T, S>(m, as, D, c, s, ln);
    } else {
      int P = 0;
      const T* pa = tt_parts<T, S>(as, D, c, tid, nt, stg, P);
      for (int s = wv; s < S; s += nw) rt_tsolve<T, S>(m, as, D, c, s, ln, tl, td, tq, pa, P);
    }
    __syncthreads();
    phase_tsolve<T, S, RES, false>(as, D, c, tid, nt, gmin, stg);
  };
  solve();
  for (int q = tid; q < 2 * nb * S; q += nt) c.dx[q] = double(c.y[q]);
  __syncthreads();
  if (sizeof(T) == 4) {
    for (int r = 0; r < kp.refine; ++r) {
      phase_adj_residual_s<T, S>(m, D, c, tid, nt, c.dx, c.F, true);
      solve();
      for (int q = tid; q < 2 * nb * S; q += nt) c.dx[q] += double(c.y[q]);
      __syncthreads();
    }
  }
  if (eval) {
    for (int idx = tid; idx < n * S; idx += nt) {
      const int i = idx / S, s = idx % S;
      const int b = slice * S + s;
      const int a = m.bus_blk[i];
      if (b >= kp.count || a < 0) continue;
      double* o = kp.out + (size_t)b * D.nj;
      o[m.ord_p[i]] = c.dx[sP<S>(a, s)];
      if (m.bus_type[i] == 0) o[D.npvpq + m.ord_q[i]] = c.dx[sP<S>(a, s) + 1];
    }
    return;
  }
  // J3^T lam via the transposed product at the solution (-(J3^T lam) lands in aux)
  // (with Step-2 weights the same product also carries vbar2 on |V| of x)
  phase_adj_residual_s<T, S>(m, D, c, tid, nt, c.dx, nullptr, false, gw);
  for (int idx = tid; idx < n * S; idx += nt) {
    const int i = idx / S, s = idx % S;
    const int b = slice * S + s;
    if (b >= kp.count) continue;
    const size_t o = (size_t)b * n + i;
    const int a = m.bus_blk[i];
    const int bt = m.bus_type[i];
    double gpd = 0.0, gqd = 0.0, gpg = 0.0, gvs = 0.0;
    if (s_ok[s]) {
      if (a >= 0) {
        gpd = c.dx[sP<S>(a, s)];
        if (bt == 0) gqd = c.dx[sP<S>(a, s) + 1];
        if (bt == 1) gpg = -c.dx[sP<S>(a, s)];
      }
      if (bt != 0) gvs = kp.g_vm[o] + c.aux[idx];
      gen_direct(kp, o, bt, gpd, gqd, gpg);
    }
    if (kp.g_pd) kp.g_pd[o] = gpd;
    if (kp.g_qd) kp.g_qd[o] = gqd;
    if (kp.g_pg) kp.g_pg[o] = gpg;
    if (kp.g_vset) kp.g_vset[o] = gvs;
  }
}

// ----------------------------------------------------------------------------
// Step 2 of the forward completion: the generation block of y at a given
// solution.  One thread per (scenario, bus); PQ rows write zeros.  The
// calculated injection of a PV or slack row is one Y_bus row product in FP64,
// with the voltages of its neighbours formed from (|V|, theta) on the fly.

__global__ void __launch_bounds__(256) k_recover(KParams kp) {
  const Sym m = bind_sym(kp.sym, kp.sym, kp.so);
  const int n = kp.dims.n_bus;
  const size_t o = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= (size_t)kp.count * n) return;
  const size_t row = o - o % n;
  const int i = (int)(o % n);
  const int bt = m.bus_type[i];
  double po = 0.0, qo = 0.0;
  if (bt != 0) {
    const double* vm = kp.vm_in + row;
    const double* va = kp.va_in + row;
    double ir = 0.0, ii = 0.0;
    for (int q = m.y_rp[i]; q < m.y_rp[i + 1]; ++q) {
      const int j = m.y_ci[q];
      double sn, cs;
      sincos(va[j], &sn, &cs);
      const double ej = vm[j] * cs, fj = vm[j] * sn;
      ir += m.y_g[q] * ej - m.y_b[q] * fj;
      ii += m.y_g[q] * fj + m.y_b[q] * ej;
    }
    double sn, cs;
    sincos(va[i], &sn, &cs);
    const double e = vm[i] * cs, f = vm[i] * sn;
    const double P = e * ir + f * ii, Q = f * ir - e * ii;   // S = V conj(I)
    qo = Q + kp.qd[o];
    po = bt == 2 ? P + kp.pd[o] : (kp.pg ? kp.pg[o] : 0.0);
  }
  if (kp.pg_out) kp.pg_out[o] = po;
  if (kp.qg_out) kp.qg_out[o] = qo;
}

// ----------------------------------------------------------------------------
// dense J1 export in the paper's ordering (evaluation entry point)

__global__ void __launch_bounds__(256) k_jacobian_dense(KParams kp) {
  const Dims& D = kp.dims;
  const Sym m = bind_sym(kp.sym, kp.sym, kp.so);
  const int b = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = D.n_bus, nj = D.nj;
  const size_t io = (size_t)b * n;
  double* gd = kp.ws_d + (size_t)b * kp.lay.sd;
  double *e = gd + kp.lay.o_e, *f = gd + kp.lay.o_f, *vm = gd + kp.lay.o_vm;
  double *ire = gd + kp.lay.o_ire, *iim = gd + kp.lay.o_iim;
  const int gk = kp.lay.gk;   // the workspace groups a bus's values: element i at i * gk
  for (int i = tid; i < n; i += nt) {
    vm[i * gk] = kp.vm_in[io + i];
    const double va = m.bus_type[i] == 2 ? 0.0 : kp.va_in[io + i];
    e[i * gk] = vm[i * gk] * cos(va);
    f[i * gk] = vm[i * gk] * sin(va);
  }
  __syncthreads();
  for (int i = tid; i < n; i += nt) {
    double ir = 0.0, ii = 0.0;
    for (int q = m.y_rp[i]; q < m.y_rp[i + 1]; ++q) {
      const int j = m.y_ci[q];
      ir += m.y_g[q] * e[j * gk] - m.y_b[q] * f[j * gk];
      ii += m.y_g[q] * f[j * gk] + m.y_b[q] * e[j * gk];
    }
    ire[i * gk] = ir;
    iim[i * gk] = ii;
  }
  __syncthreads();
  double* o = kp.out + (size_t)b * nj * nj;
  for (size_t q = tid; q < (size_t)nj * nj; q += nt) o[q] = 0.0;
  __syncthreads();
  for (int i = tid; i < n; i += nt) {
    if (m.bus_type[i] == 2) continue;
    const int rP = m.ord_p[i];
    const int rQ = m.bus_type[i] == 0 ? D.npvpq + m.ord_q[i] : -1;
    for (int q = m.y_rp[i]; q < m.y_rp[i + 1]; ++q) {
      const int j = m.y_ci[q];
      if (m.bus_type[j] == 2) continue;
      const J4 x = (i == j) ? jac_diag(m.y_g[q], m.y_b[q], e[i * gk], f[i * gk], vm[i * gk], 1.0 / vm[i * gk], ire[i * gk], iim[i * gk])
                            : jac_off(m.y_g[q], m.y_b[q], e[i * gk], f[i * gk], e[j * gk], f[j * gk], 1.0 / vm[j * gk]);
      const int cT = D.npq + m.ord_p[j];
      const int cV = m.bus_type[j] == 0 ? m.ord_q[j] : -1;
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
static hipError_t launch_newton_t(const KParams& kp, int slice, int grid, int nt, size_t lds,
                                  bool res, hipStream_t st) {
  dim3 g(grid), b(nt);
  if (res && (nt != res_newton_threads<T>() || slice > kResMaxSlice)) return hipErrorInvalidValue;
  if (!res) {
    switch (slice) {
      case 1: hipLaunchKernelGGL((k_newton<T, false, 1>), g, b, lds, st, kp); break;
      case 2: hipLaunchKernelGGL((k_newton<T, false, 2>), g, b, lds, st, kp); break;
      case 4: hipLaunchKernelGGL((k_newton<T, false, 4>), g, b, lds, st, kp); break;
      case 8: hipLaunchKernelGGL((k_newton<T, false, 8>), g, b, lds, st, kp); break;
      case 16: hipLaunchKernelGGL((k_newton<T, false, 16>), g, b, lds, st, kp); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (slice) {
      case 1: hipLaunchKernelGGL((k_newton<T, true, 1>), g, b, lds, st, kp); break;
      case 2: hipLaunchKernelGGL((k_newton<T, true, 2>), g, b, lds, st, kp); break;
      case 4: hipLaunchKernelGGL((k_newton<T, true, 4>), g, b, lds, st, kp); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_newton(const KParams& kp, bool fp32, int slice, int grid, int nt, size_t lds,
                         bool lds_res, hipStream_t st) {
  return fp32 ? launch_newton_t<float>(kp, slice, grid, nt, lds, lds_res, st)
              : launch_newton_t<double>(kp, slice, grid, nt, lds, lds_res, st);
}

template <typename T>
static hipError_t launch_adjoint_hbm_t(const KParams& kp, int slice, int grid, int nt, size_t lds, hipStream_t st);

template <typename T>
static hipError_t launch_adjoint_t(const KParams& kp, int slice, int grid, int nt, size_t lds, hipStream_t st) {
  if (slice < 0) return launch_adjoint_hbm_t<T>(kp, -slice, grid, nt, lds, st);
  if (nt != kResThreads) return hipErrorInvalidValue;
  switch (slice) {
    case 1: hipLaunchKernelGGL((k_adjoint_slice<T, true, 1>), dim3(grid), dim3(nt), lds, st, kp); break;
    case 2: hipLaunchKernelGGL((k_adjoint_slice<T, true, 2>), dim3(grid), dim3(nt), lds, st, kp); break;
    case 4: hipLaunchKernelGGL((k_adjoint_slice<T, true, 4>), dim3(grid), dim3(nt), lds, st, kp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_adjoint_hbm_t(const KParams& kp, int slice, int grid, int nt, size_t lds, hipStream_t st) {
  if (nt > 1024) return hipErrorInvalidValue;
  switch (slice) {
    case 1: hipLaunchKernelGGL((k_adjoint_slice<T, false, 1>), dim3(grid), dim3(nt), lds, st, kp); break;
    case 2: hipLaunchKernelGGL((k_adjoint_slice<T, false, 2>), dim3(grid), dim3(nt), lds, st, kp); break;
    case 4: hipLaunchKernelGGL((k_adjoint_slice<T, false, 4>), dim3(grid), dim3(nt), lds, st, kp); break;
    case 8: hipLaunchKernelGGL((k_adjoint_slice<T, false, 8>), dim3(grid), dim3(nt), lds, st, kp); break;
    case 16: hipLaunchKernelGGL((k_adjoint_slice<T, false, 16>), dim3(grid), dim3(nt), lds, st, kp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(const KParams& kp, bool fp32, int slice, int grid, int nt, size_t lds, hipStream_t st) {
  return fp32 ? launch_adjoint_t<float>(kp, slice, grid, nt, lds, st)
              : launch_adjoint_t<double>(kp, slice, grid, nt, lds, st);
}

hipError_t launch_recover(const KParams& kp, hipStream_t st) {
  const size_t total = (size_t)kp.count * kp.dims.n_bus;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_recover, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, kp);
  return hipGetLastError();
}

hipError_t launch_jacobian_dense(const KParams& kp, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobian_dense, dim3(grid), dim3(256), 0, st, kp);
  return hipGetLastError();
}

template <typename T>
static hipError_t set_lds_t(int max_lds) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* fn) {
    hipError_t r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (r != hipSuccess) e = r;
  };
  set(reinterpret_cast<const void*>(&k_newton<T, false, 1>));
  set(reinterpret_cast<const void*>(&k_newton<T, false, 2>));
  set(reinterpret_cast<const void*>(&k_newton<T, false, 4>));
  set(reinterpret_cast<const void*>(&k_newton<T, false, 8>));
  set(reinterpret_cast<const void*>(&k_newton<T, false, 16>));
  set(reinterpret_cast<const void*>(&k_newton<T, true, 1>));
  set(reinterpret_cast<const void*>(&k_newton<T, true, 2>));
  set(reinterpret_cast<const void*>(&k_newton<T, true, 4>));
  set(reinterpret_cast<const void*>(&k_adjoint_slice<T, true, 1>));
  set(reinterpret_cast<const void*>(&k_adjoint_slice<T, true, 2>));
  set(reinterpret_cast<const void*>(&k_adjoint_slice<T, true, 4>));
  set(reinterpret_cast<const void*>(&k_adjoint_slice<T, false, 1>));
  set(reinterpret_cast<const void*>(&k_adjoint_slice<T, false, 2>));
  set(reinterpret_cast<const void*>(&k_adjoint_slice<T, false, 4>));
  set(reinterpret_cast<const void*>(&k_adjoint_slice<T, false, 8>));
  set(reinterpret_cast<const void*>(&k_adjoint_slice<T, false, 16>));
  return e;
}

hipError_t read_phase_clocks(unsigned long long* ticks, int n, bool reset) {
#ifdef SABLE_PHASE_CLOCKS
  if (n > kPhaseSlots) n = kPhaseSlots;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && n > 0) e = hipMemcpyFromSymbol(ticks, HIP_SYMBOL(g_phase_ticks), n * sizeof(unsigned long long));
  if (e == hipSuccess && reset) {
    unsigned long long zero[kPhaseSlots] = {};
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_phase_ticks), zero, sizeof(zero));
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  return e;
#else
  (void)ticks; (void)n; (void)reset;
  return hipErrorNotSupported;
#endif
}

hipError_t set_lds_limits(size_t max_lds) {
  hipError_t e1 = set_lds_t<double>((int)max_lds);
  hipError_t e2 = set_lds_t<float>((int)max_lds);
  return e1 != hipSuccess ? e1 : e2;
}

}  // namespace sable
