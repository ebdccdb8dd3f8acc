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
  MODE_EVAL_FILL = 5,      // the Jacobian values in the LU positions, before factorisation
};

// slots of the per-phase wall-clock counters (builds with
// -DSABLE_PHASE_CLOCKS): ticks of the Newton kernel's phases, then event
// counts; accumulated over launches by workgroup 0
enum PhaseSlot : int {
  PH_SETUP = 0,                // inputs, flat start
  PH_MISMATCH = 1,             // I = Y V, F1, norms and the convergence test
  PH_FILL = 2,                 // Jacobian values into the LU positions (Algorithm 1)
  PH_FACTOR_LEVELS = 3,        // level-scheduled factorisation with the fused forward solve
  PH_FACTOR_TAIL = 4,          // dense tail factorisation (+ its forward solve)
  PH_BSOLVE_TAIL = 5,          // backward solve of the tail rows
  PH_BSOLVE_LEVELS = 6,        // level-scheduled backward solve
  PH_REFINE_DV = 7,            // refinement: dV from the correction
  PH_REFINE_RESIDUAL = 8,      // refinement: FP64 residual through Y_bus
  PH_REFINE_FSOLVE_LEVELS = 9, // refinement: level-scheduled forward solve
  PH_REFINE_TAIL = 10,         // refinement: tail forward + backward solves
  PH_REFINE_BSOLVE_LEVELS = 11,// refinement: level-scheduled backward solve
  PH_OTHER = 12,               // copies of the correction, state update, e + jf
  PH_KEEP = 13,                // refresh and refactorisation at the solution (kept factors)
  PH_OUTPUT = 14,              // outputs
  PH_NEWTON_LAUNCHES = 16,     // count: launches
  PH_NEWTON_STEPS = 17,        // count: Newton corrections of workgroup 0
  PH_REFINE_STEPS = 18,        // count: refinement steps of workgroup 0
  kPhaseSlots = 32
};

// LDS scratch at the start of every kernel's dynamic LDS: per-(wave,
// scenario) partial maxima and flags, per-scenario reductions, zero-pivot
// flags and Newton bookkeeping (iterations, status, final mismatch).
constexpr int kMaxWaves = 16;
constexpr int kMaxSlice = 16;
constexpr int kRedOff = 0;                                     // double [16][16]
constexpr int kFlagOff = kRedOff + 8 * kMaxWaves * kMaxSlice;  // int [16][16]
constexpr int kPivOff = kFlagOff + 4 * kMaxWaves * kMaxSlice;  // int [16]
constexpr int kFnOff = kPivOff + 4 * kMaxSlice;                // double [16]
constexpr int kBadOff = kFnOff + 8 * kMaxSlice;                // int [16]
constexpr int kItOff = kBadOff + 4 * kMaxSlice;                // int [16]
constexpr int kStOff = kItOff + 4 * kMaxSlice;                 // int [16]
constexpr int kFnvOff = kStOff + 4 * kMaxSlice;                // double [16]
constexpr int kScratchBytes = 4096;
static_assert(kFnvOff + 8 * kMaxSlice <= kScratchBytes, "scratch layout");

// Byte offsets of the symbolic arrays inside one packed image (device
// memory; the prefix [0, newton_bytes) is what the Newton kernel reads and is
// copied whole into LDS when the slice of a workgroup is LDS-resident).
struct SymOffsets {
  int bus_type, bus_blk, y_rp, y_ci, y_g, y_b;
  int rp, ci, diag, fill4, tail_pos, tail_split, tail_mask;
  int f_ptr, f_blob, fs_ptr, fs_blob, bs_ptr, bs_blob;   // level metadata chunks
  int newton_bytes;
  // [newton_bytes, adj_bytes): what the LDS-resident adjoint reads besides
  int ut_ptr, ut_blob, lt_ptr, lt_blob, tt_ptr, tt_pairs, y_tr;
  int adj_bytes;
  int tail_cblk;                          // position of each compact tail block (LDS copy of the tail)
  int tail_prog;                          // per-pivot elimination program of the tail (LDS tail copy)
  int ord_p, ord_q;                       // paper-order positions (exports)
  int total_bytes;
};

struct Dims {
  int n_bus, nb, nnzb, nj, npq, npvpq;
  int nlev_l, nlev_u;             // full level schedules (adjoint)
  int nlev_f, nlev_fs, nlev_bs;   // factor-task, forward and backward levels outside the tail
  int tail_t, tail_base;          // dense tail rows [tail_base, tail_base + tail_t)
  int nch_f, nch_fs, nch_bs;      // metadata chunks of the factor, forward and backward levels
  int nch_ut, nch_lt;             // metadata chunks of the transposed solves
  int chunk_ints;                 // largest chunk (int32 words), staged after the LDS scratch
  int tail_nblk;                  // blocks of the tail rows in tail columns (LDS tail copy)
  int tail_nbs;                  // stride of a scenario's blocks in the LDS tail copy (odd)
  int tail_prog_ints;             // words of the tail program
  int tail_prog_prefix;           // its records, step and column words: kept in LDS
  int tail_prog_lds;              // 1: its update words staged in the metadata area, 0: read in place
  int y_lds_off;                  // HBM-resident slices: byte offset of y in LDS (0: y stays in HBM)
};

// Offsets of the per-scenario arrays, in elements.  FP64 arrays:
// e f vm va ire iim ps qs dvr dvi aux rvm (= 1/|V|) [n_bus], F dx [2 nb].  Factor-
// precision arrays (T): y [2 nb], lu [4 nnzb], dinv [4 nb].  In a slice of S
// scenarios every array is interleaved by scenario (element k of scenario s
// at k*S + s) and starts at offset*S, except that with gk = 8 (gk = 2) the
// eight gathered per-bus values e f vm rvm ire iim dvr dvi are grouped by bus
// (in the pairs e f, vm rvm, ire iim, dvr dvi): the grouped offsets are
// consecutive and bus i of scenario s sits at i*gk*S + s past them.
struct StateLayout {
  int o_e, o_f, o_vm, o_va, o_ire, o_iim, o_ps, o_qs, o_dvr, o_dvi, o_aux, o_rvm, o_F, o_dx;
  int gk;  // 8: the eight per-bus values grouped, 2: in pairs, 1: one array each
  int sd;  // doubles per scenario
  int o_y, o_lu, o_dinv;
  int st;  // T elements per scenario
};

struct KParams {
  Dims dims;
  SymOffsets so;
  const unsigned char* sym;  // packed symbolic image (device)
  StateLayout lay;           // per-scenario layout of the HBM workspace
  StateLayout llay;          // per-scenario layout inside an LDS-resident slice
  StateLayout alay;          // per-scenario layout inside an LDS-resident adjoint slice
  double* ws_d;              // per-scenario workspace (layout lay)
  void* ws_t;
  int* ws_i;
  double* wsl_d;             // HBM-resident slices: S scenarios interleaved per slice
  void* wsl_t;
  int mode, max_iter, refine, adaptive, keep, count, gmin, wstride;
  double tol;
  const double *pd, *qd, *pg, *vset, *vm_in, *va_in, *rhs, *g_vm, *g_va;
  double *vm_out, *va_out, *fnorm_out, *out, *g_pd, *g_qd, *g_pg, *g_vset;
  int *iters_out, *status_out;
  // Step 2: recovered generation (outputs) and the loss's gradients on it
  // (inputs of the completed adjoint); [batch][n_bus], any may be null
  double *pg_out, *qg_out;
  const double *g_pgo, *g_qgo;
};

// LDS-resident slices: one wavefront per scenario for the register-resident
// dense tail, at most 4 scenarios per workgroup.  The Newton kernel and the
// adjoint run kResThreads: the wavefronts beyond the slice's tails hide LDS
// latency in the barrier-separated phases (with FP64 factors the register
// tail then fits the 256 registers a 512-thread workgroup leaves a
// wavefront with a few spilled values outside the inner loops).
constexpr int kResThreads = 512;
constexpr int kResMaxSlice = 4;
template <typename T>
constexpr int res_newton_threads() { return kResThreads; }
inline int res_newton_threads(bool) { return kResThreads; }

// slice = scenarios per workgroup: 1, 2 or 4 when LDS-resident, up to 16 otherwise.
hipError_t launch_newton(const KParams& kp, bool fp32, int slice, int grid, int nt, size_t lds,
                         bool lds_res, hipStream_t st);
// slice > 0: LDS-resident adjoint slices of that width (kResThreads threads);
// slice < 0: HBM-resident slices of width -slice reading the forward solve's
// slice workspace (at most 1024 threads)
hipError_t launch_adjoint(const KParams& kp, bool fp32, int slice, int grid, int nt, size_t lds, hipStream_t st);
hipError_t launch_jacobian_dense(const KParams& kp, int grid, hipStream_t st);
// Step-2 recovery of the generation block for kp.count scenarios
hipError_t launch_recover(const KParams& kp, hipStream_t st);
hipError_t set_lds_limits(size_t max_lds);
// copies (and optionally clears) the per-phase counters; hipErrorNotSupported
// when the library was built without them
hipError_t read_phase_clocks(unsigned long long* ticks, int n, bool reset);

}  // namespace sable
