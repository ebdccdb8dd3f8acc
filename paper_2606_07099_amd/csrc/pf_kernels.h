// Device-side data structures and launchers shared by the C-ABI layer and
// the kernels.  Plain pointers and sizes only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sable {

enum Mode : int {
  MODE_SOLVE = 0,          // Newton from the flat start
  MODE_EVAL_MISMATCH = 1,  // F1 at a given state
  MODE_EVAL_STEP = 2,      // Newton correction at a given state
  MODE_EVAL_FACTOR = 3,    // factor J1 at a given state and keep it
  MODE_EVAL_ADJOINT = 4,   // adjoint solve with a given right-hand side
};

// LDS scratch at the start of every kernel's dynamic LDS
constexpr int kRedBytes = 8 * 32;            // per-wave partial maxima
constexpr int kFlagInts = 64;                // per-wave flags + zero-pivot flag
constexpr int kZeroPivotFlag = 32;
constexpr int kScratchBytes = kRedBytes + 4 * kFlagInts;

// Symbolic arrays on the device (one allocation, see pf_api.cpp).
struct DevSym {
  int n_bus, nb, nnzb, nj, npq, npvpq, nlev_l, nlev_u;
  const int *bus_type, *bus_blk, *blk_bus, *ord_p, *ord_q;
  const int *y_rp, *y_ci, *y_tr;
  const double *y_g, *y_b;
  const int *rp, *ci, *diag, *mirror, *lu_src, *upd_start, *upd_tgt;
  const int *lev_l_ptr, *lev_l_rows, *lev_u_ptr, *lev_u_rows;
};

// Offsets of the per-scenario arrays.  FP64 arrays (in units of double):
// e f vm va ire iim ps qs dvr dvi aux [n_bus], F dx rr [2 nb].  Factor-
// precision arrays (units of T): y [2 nb], lu [4 nnzb], dinv [4 nb].
struct StateLayout {
  int o_e, o_f, o_vm, o_va, o_ire, o_iim, o_ps, o_qs, o_dvr, o_dvi, o_aux, o_F, o_dx, o_rr;
  int sd;  // doubles per scenario
  int o_y, o_lu, o_dinv;
  int st;  // T elements per scenario
};

struct KParams {
  DevSym s;
  StateLayout lay;
  double* ws_d;
  void* ws_t;
  int* ws_i;
  int mode, max_iter, refine, keep, count, gmin, wstride;
  double tol;
  const double *pd, *qd, *pg, *vset, *vm_in, *va_in, *rhs, *g_vm, *g_va;
  double *vm_out, *va_out, *fnorm_out, *out, *g_pd, *g_qd, *g_pg, *g_vset;
  int *iters_out, *status_out;
};

hipError_t launch_newton(const KParams& kp, bool fp32, int grid, int nt, size_t lds, bool lds_res,
                         hipStream_t st);
hipError_t launch_adjoint(const KParams& kp, bool fp32, int grid, int nt, hipStream_t st);
hipError_t launch_jacobian_dense(const KParams& kp, int grid, hipStream_t st);
hipError_t set_lds_limits(size_t max_lds);

}  // namespace sable
