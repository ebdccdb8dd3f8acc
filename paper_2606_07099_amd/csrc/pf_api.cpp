// C-ABI of the batched Newton power-flow library (declared in sable_pf.h).
//
// pf_template_build runs the host symbolic analysis once, uploads the shared
// pattern, schedules and fill map in one device allocation, and allocates the
// per-scenario workspace for the whole batch; solve / adjoint calls only
// enqueue kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "operators.h"
#include "pf_kernels.h"
#include "pf_operators.h"
#include "sable_pf.h"
#include "symbolic.h"

struct pf_template {
  sable::Symbolic sym;
  pf_options opt{};
  int32_t batch = 0;
  bool fp32 = false;
  int nt = 256;
  bool lds_res = false;
  size_t lds_bytes = 0;
  int gmin = 4;
  int wstride = 0;
  int slice = 1;             // scenarios per workgroup
  int device = 0;
  sable::StateLayout lay{};  // HBM workspace, per scenario
  sable::StateLayout llay{}; // inside an LDS-resident slice, per scenario
  sable::StateLayout alay{}; // inside an LDS-resident adjoint slice, per scenario
  int adj_slice = 0;         // > 0: LDS-resident adjoint slices of this width, < 0: HBM-resident
  int adj_nt = 256;
  size_t adj_lds = 0;
  sable::SymOffsets so{};
  sable::Dims dims{};
  void* d_sym = nullptr;
  double* ws_d = nullptr;
  void* ws_t = nullptr;
  int* ws_i = nullptr;
  double* wsl_d = nullptr;   // HBM-resident slices of S > 1 scenarios
  void* wsl_t = nullptr;
  size_t ws_bytes = 0;
  bool have_factors = false;
  // operator export tables, built with the template: the base entries
  // (int4 each), then per operator its source map, CSR row pointers and
  // column indices (one scenario's pattern)
  void* d_ops = nullptr;
  int32_t op_nbase = 0;
  int32_t op_off[sable::OP_COUNT] = {};
  int32_t op_nnz[sable::OP_COUNT] = {};
  int32_t op_ip_off[sable::OP_COUNT] = {};
  int32_t op_ix_off[sable::OP_COUNT] = {};
  int32_t op_rows[sable::OP_COUNT] = {};
  int32_t op_cols[sable::OP_COUNT] = {};
  double* d_opef = nullptr;   // per-bus state (e, f, P, Q) of the last operator refresh
  size_t opef_count = 0;      // scenarios it holds
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return PF_EHIP;
}

// keeps the caller's current device, switches to the template's for a call
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() { if (prev >= 0) (void)hipSetDevice(prev); }
};

// largest level-metadata chunk an HBM-resident workgroup stages in LDS
// (int32 words; 48 KB)
constexpr int32_t kChunkInts = 12288;

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// HBM workspace of a scenario (also the layout of the interleaved slice
// workspace).  grouped: the eight per-bus values that the gathers read (e f
// |V| 1/|V| I_re I_im dV_re dV_im) sit together by bus, so that a gather of a
// bus reads one run per scenario instead of one per value.  That pays off for
// slices of several scenarios, whose bus-order passes still read whole runs;
// a slice of one scenario keeps one array per value, so that its bus-order
// passes read consecutive buses of one array.
// gk: how the eight gathered values e f |V| 1/|V| I_re I_im dV_re dV_im of a
// bus are grouped: 8 all together, 2 in the pairs (e, f), (|V|, 1/|V|),
// (I_re, I_im), (dV_re, dV_im) that the passes read together, 1 one array each
sable::StateLayout make_layout(int n_bus, int nb, int nnzb, int gk) {
  sable::StateLayout L{};
  const int nbr = round_up(n_bus, 4), v2 = round_up(2 * nb, 4);
  int o = 0;
  L.gk = gk;
  int* fld[8] = {&L.o_e, &L.o_f, &L.o_vm, &L.o_rvm, &L.o_ire, &L.o_iim, &L.o_dvr, &L.o_dvi};
  for (int k = 0; k < 8; ++k)
    *fld[k] = o + (gk == 8 ? k : gk == 2 ? (k >> 1) * 2 * nbr + (k & 1) : k * nbr);
  o += 8 * nbr;
  L.o_va = o; o += nbr; L.o_ps = o; o += nbr; L.o_qs = o; o += nbr; L.o_aux = o; o += nbr;
  L.o_F = o; o += 2 * nbr; L.o_dx = o; o += v2;   // F by bus, dx by block row
  L.sd = o;
  int t = 0;
  L.o_y = t; t += round_up(2 * nb, 8);
  L.o_lu = t; t += round_up(4 * nnzb, 8);
  L.o_dinv = t; t += round_up(4 * nb, 8);
  L.st = t;
  return L;
}

// compact per-scenario layout inside an LDS-resident slice: the refinement
// vectors only exist in the mixed-precision mode, the adjoint scratch never
sable::StateLayout make_lds_layout(int n_bus, int nb, int nnzb, bool mixed) {
  sable::StateLayout L{};
  L.gk = 1;
  int o = 0;
  L.o_e = o; o += n_bus; L.o_f = o; o += n_bus; L.o_vm = o; o += n_bus; L.o_va = o; o += n_bus;
  L.o_ire = o; o += n_bus; L.o_iim = o; o += n_bus; L.o_ps = o; o += n_bus; L.o_qs = o; o += n_bus;
  L.o_rvm = o; o += n_bus;
  L.o_F = o; o += 2 * n_bus; L.o_dx = o; o += 2 * nb;
  if (mixed) {
    L.o_dvr = o; o += n_bus; L.o_dvi = o; o += n_bus;
  } else {
    L.o_dvr = L.o_dvi = 0;
  }
  L.o_aux = 0;
  L.sd = round_up(o, 2);
  int t = 0;
  L.o_y = t; t += round_up(2 * nb, 4);   // blocks start 16-byte aligned
  L.o_lu = t; t += 4 * nnzb;
  L.o_dinv = t; t += 4 * nb;
  L.st = round_up(t, 4);
  return L;
}

// per-scenario layout inside an LDS-resident adjoint slice: the kept state
// (e f |V|), the currents, the adjoint scratch and the factors
sable::StateLayout make_adj_layout(int n_bus, int nb, int nnzb) {
  sable::StateLayout L{};
  L.gk = 1;
  int o = 0;
  L.o_e = o; o += n_bus; L.o_f = o; o += n_bus; L.o_vm = o; o += n_bus;
  L.o_ire = o; o += n_bus; L.o_iim = o; o += n_bus;
  L.o_dvr = o; o += n_bus; L.o_dvi = o; o += n_bus; L.o_aux = o; o += n_bus;
  L.o_F = o; o += 2 * n_bus; L.o_dx = o; o += 2 * nb;
  L.o_va = L.o_ps = L.o_qs = L.o_rvm = 0;
  L.sd = round_up(o, 2);
  int t = 0;
  L.o_y = t; t += round_up(2 * nb, 4);   // blocks start 16-byte aligned
  L.o_lu = t; t += 4 * nnzb;
  L.o_dinv = t; t += 4 * nb;
  L.st = round_up(t, 4);
  return L;
}

// packs int32 / double host arrays into one device buffer
struct Packer {
  std::vector<unsigned char> buf;
  size_t align() {
    buf.resize((buf.size() + 15) / 16 * 16);
    return buf.size();
  }
  template <typename V>
  size_t add(const std::vector<V>& v) {
    size_t off = (buf.size() + 15) / 16 * 16;
    buf.resize(off + v.size() * sizeof(V));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(V));
    return off;
  }
};

void fill_stats(const sable::Symbolic& S, pf_template_stats* o) {
  std::memset(o, 0, sizeof(*o));
  o->n_bus = S.n_bus;
  o->n_pv = S.n_pv;
  o->n_pq = S.n_pq;
  o->n_j = S.nb + S.n_pq;
  o->nnz_ybus = (int32_t)S.y_ci.size();
  o->nnz_j1 = S.nnz_j1;
  o->n_blocks = S.nb;
  o->nnzb_lu = S.nnzb();
  o->nnz_lu = S.nnz_lu;
  o->n_block_updates = S.n_upd;
  o->n_levels_l = S.n_levels_l();
  o->n_levels_u = S.n_levels_u();
  o->max_row_blocks = S.max_row_blocks;
  o->fill_ratio = S.nnz_j1 > 0 ? (double)S.nnz_lu / (double)S.nnz_j1 : 0.0;
  o->factor_flops = S.factor_flops;
}

bool structurally_symmetric(const sable::Symbolic& S) {
  for (int32_t q : S.y_tr) if (q < 0) return false;
  return true;
}

sable::KParams base_params(const pf_template* t) {
  sable::KParams kp{};
  kp.dims = t->dims;
  kp.so = t->so;
  kp.sym = static_cast<const unsigned char*>(t->d_sym);
  kp.lay = t->lay;
  kp.llay = t->llay;
  kp.alay = t->alay;
  kp.ws_d = t->ws_d ? t->ws_d : t->wsl_d;   // wide HBM-resident slices: the slice workspace
  kp.ws_t = t->ws_t ? t->ws_t : t->wsl_t;   // serves as per-scenario scratch
  kp.ws_i = t->ws_i;
  kp.wsl_d = t->wsl_d ? t->wsl_d : t->ws_d;
  kp.wsl_t = t->wsl_t ? t->wsl_t : t->ws_t;
  kp.max_iter = t->opt.max_iter;
  kp.refine = t->fp32 ? t->opt.refine_steps : 0;
  kp.adaptive = t->opt.refine_adaptive;
  kp.keep = t->opt.keep_factors;
  kp.gmin = t->gmin;
  kp.wstride = t->wstride;
  kp.tol = t->opt.tol;
  kp.count = t->batch;
  return kp;
}

// the operator tables of a template: one device buffer of int32
int build_operator_tables(pf_template* t) {
  const sable::Symbolic& S = t->sym;
  sable::OperatorSet ops;
  std::string err;
  const int rc = sable::build_operators(S.n_bus, S.bus_type.data(), S.y_rp.data(), S.y_ci.data(), ops, err);
  if (rc != PF_OK) return fail(rc, "operator tables: " + err);
  std::vector<int32_t> buf;
  for (const sable::BaseEntry& e : ops.base) buf.insert(buf.end(), {e.kind, e.i, e.j, e.q});
  t->op_nbase = (int32_t)ops.base.size();
  for (int k = 0; k < sable::OP_COUNT; ++k) {
    const sable::OperatorPattern& op = ops.op[k];
    t->op_off[k] = (int32_t)buf.size();
    t->op_nnz[k] = (int32_t)op.src.size();
    buf.insert(buf.end(), op.src.begin(), op.src.end());
    t->op_ip_off[k] = (int32_t)buf.size();
    buf.insert(buf.end(), op.indptr.begin(), op.indptr.end());
    t->op_ix_off[k] = (int32_t)buf.size();
    buf.insert(buf.end(), op.indices.begin(), op.indices.end());
    t->op_rows[k] = op.rows;
    t->op_cols[k] = op.cols;
  }
  void* d = nullptr;
  if (hipMalloc(&d, buf.size() * sizeof(int32_t)) != hipSuccess)
    return fail(PF_ENOMEM, "pf_template_build: device allocation (operator tables)");
  hipError_t he = hipMemcpy(d, buf.data(), buf.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(he, "pf_template_build: operator table upload");
  }
  t->d_ops = d;
  t->ws_bytes += buf.size() * sizeof(int32_t);
  return PF_OK;
}

int adjoint_impl(const char* name, pf_template* t, const double* g_vm, const double* g_va,
                 const double* g_pgo, const double* g_qgo, double* g_pd, double* g_qd, double* g_pg,
                 double* g_vset, void* hip_stream) {
  g_err.clear();
  const std::string nm(name);
  if (!t) return fail(PF_EINVAL, nm + ": template is NULL");
  if (!g_vm || !g_va) return fail(PF_EINVAL, nm + ": NULL gradient input");
  if (!t->have_factors)
    return fail(PF_ESTATE, nm + ": needs a preceding pf_solve_batch with keep_factors=1");
  DeviceGuard g(t->device);
  sable::KParams kp = base_params(t);
  kp.mode = sable::MODE_SOLVE;
  kp.g_vm = g_vm; kp.g_va = g_va;
  kp.g_pgo = g_pgo; kp.g_qgo = g_qgo;
  kp.g_pd = g_pd; kp.g_qd = g_qd; kp.g_pg = g_pg; kp.g_vset = g_vset;
  const int aw = t->adj_slice < 0 ? -t->adj_slice : t->adj_slice;
  const int agrid = aw ? (t->batch + aw - 1) / aw : t->batch;
  hipError_t he = sable::launch_adjoint(kp, t->fp32, t->adj_slice, agrid, aw ? t->adj_nt : t->nt, t->adj_lds,
                                        static_cast<hipStream_t>(hip_stream));
  if (he != hipSuccess) return hip_fail(he, (nm + ": launch").c_str());
  return PF_OK;
}

}  // namespace

namespace sable {

void set_error(const std::string& msg) { g_err = msg; }

int operator_params(pf_template* t, int which, int count, const double* vm, const double* va, double* values,
                    const char* name, OpParams& p, int& device) {
  g_err.clear();
  const std::string nm(name);
  if (!t) return fail(PF_EINVAL, nm + ": template is NULL");
  if (which < 0 || which >= OP_COUNT) return fail(PF_EINVAL, nm + ": unknown operator");
  if (count < 0) return fail(PF_EINVAL, nm + ": negative count");
  if (count > 0 && (!vm || !va || !values)) return fail(PF_EINVAL, nm + ": NULL array");
  const unsigned char* img = static_cast<const unsigned char*>(t->d_sym);
  p = OpParams{};
  p.base = static_cast<const int4*>(t->d_ops);
  p.src = static_cast<const int*>(t->d_ops) + t->op_off[which];
  p.y_rp = reinterpret_cast<const int*>(img + t->so.y_rp);
  p.y_ci = reinterpret_cast<const int*>(img + t->so.y_ci);
  p.y_g = reinterpret_cast<const double*>(img + t->so.y_g);
  p.y_b = reinterpret_cast<const double*>(img + t->so.y_b);
  p.vm = vm;
  p.va = va;
  p.values = values;
  p.nnz = t->op_nnz[which];
  p.n_bus = t->sym.n_bus;
  p.count = count;
  device = t->device;
  return PF_OK;
}

}  // namespace sable

extern "C" {

void pf_default_options(pf_options* opt) {
  if (!opt) return;
  opt->tol = 1e-8;
  opt->max_iter = 20;
  opt->precision = PF_FP64;
  opt->refine_steps = 2;
  opt->refine_adaptive = 0;
  opt->keep_factors = 1;
  opt->block_threads = 0;
}

const char* pf_last_error(void) { return g_err.c_str(); }

int pf_ybus_from_branches(int32_t n_bus, int32_t n_branch, const int32_t* from, const int32_t* to,
                          const double* r, const double* x, const double* b_charging,
                          int32_t* indptr, int32_t* indices, double* g, double* b,
                          int32_t capacity, int32_t* nnz_out) {
  g_err.clear();
  std::vector<int32_t> rp, ci;
  std::vector<double> gv, bv;
  std::string err;
  int nnz = sable::ybus_from_branches(n_bus, n_branch, from, to, r, x, b_charging, rp, ci, gv, bv, err);
  if (nnz < 0) return fail(nnz, err);
  if (nnz_out) *nnz_out = nnz;
  if (!indptr || !indices || !g || !b) return fail(PF_EINVAL, "pf_ybus_from_branches: null output array");
  if (nnz > capacity) return fail(PF_EINVAL, "pf_ybus_from_branches: capacity too small");
  std::copy(rp.begin(), rp.end(), indptr);
  std::copy(ci.begin(), ci.end(), indices);
  std::copy(gv.begin(), gv.end(), g);
  std::copy(bv.begin(), bv.end(), b);
  return PF_OK;
}

int pf_symbolic_analyze(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
                        const int32_t* y_indices, pf_template_stats* out, int32_t* bus_order) {
  g_err.clear();
  if (!out) return fail(PF_EINVAL, "pf_symbolic_analyze: out is NULL");
  if (n_bus < 2 || !y_indptr) return fail(PF_EINVAL, "pf_symbolic_analyze: bad sizes");
  const int32_t nnz = y_indptr[n_bus];
  if (nnz < 0) return fail(PF_EINVAL, "pf_symbolic_analyze: bad y_indptr");
  std::vector<double> ones(nnz, 1.0);
  sable::Symbolic S;
  std::string err;
  int rc = sable::analyze(n_bus, bus_type, y_indptr, y_indices, ones.data(), ones.data(), S, err);
  if (rc != PF_OK) return fail(rc, err);
  if (!structurally_symmetric(S)) return fail(PF_EINVAL, "Y_bus pattern must be structurally symmetric");
  fill_stats(S, out);
  if (bus_order) std::copy(S.blk_bus.begin(), S.blk_bus.end(), bus_order);
  return PF_OK;
}

int pf_template_build(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
                      const int32_t* y_indices, const double* y_g, const double* y_b,
                      int32_t batch, const pf_options* opt_in, pf_template** out) {
  g_err.clear();
  if (!out) return fail(PF_EINVAL, "pf_template_build: out is NULL");
  *out = nullptr;
  pf_options opt;
  pf_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (batch <= 0) return fail(PF_EINVAL, "pf_template_build: batch must be positive");
  if (!(opt.tol > 0.0) || opt.max_iter < 0 || (opt.precision != PF_FP64 && opt.precision != PF_MIXED) ||
      opt.refine_steps < 0 || opt.refine_steps > 16 || opt.block_threads < 0 ||
      (opt.refine_adaptive != 0 && opt.refine_adaptive != 1) ||
      opt.block_threads > 1024 || (opt.block_threads % 64) != 0)
    return fail(PF_EINVAL, "pf_template_build: invalid options");

  pf_template* t = new (std::nothrow) pf_template();
  if (!t) return fail(PF_ENOMEM, "pf_template_build: host allocation failed");
  std::string err;
  // the dense tail of an LDS-resident slice lives in registers: at most 32
  // block rows in FP32, 16 in FP64
  const int tail_max = opt.precision == PF_MIXED ? 32 : 16;
  int rc = sable::analyze(n_bus, bus_type, y_indptr, y_indices, y_g, y_b, t->sym, err, tail_max);
  if (rc != PF_OK) { delete t; return fail(rc, err); }
  if (!structurally_symmetric(t->sym)) {
    delete t;
    return fail(PF_EINVAL, "pf_template_build: Y_bus pattern must be structurally symmetric");
  }
  const sable::Symbolic& S = t->sym;
  t->opt = opt;
  t->batch = batch;
  t->fp32 = opt.precision == PF_MIXED;
  const size_t tsz = t->fp32 ? 4 : 8;

  hipError_t he = hipGetDevice(&t->device);
  if (he != hipSuccess) { delete t; return hip_fail(he, "pf_template_build: no HIP device"); }
  hipDeviceProp_t prop;
  he = hipGetDeviceProperties(&prop, t->device);
  if (he != hipSuccess) { delete t; return hip_fail(he, "pf_template_build: device query"); }
  const size_t max_lds = prop.sharedMemPerBlock;

  // ---- device symbolic image: the arrays the Newton kernel reads first
  // (copied whole into LDS by LDS-resident slices), then the rest
  std::vector<int32_t> ord_p(S.n_bus, -1), ord_q(S.n_bus, -1);
  int np = 0, nq = 0;
  for (int i = 0; i < S.n_bus; ++i) {
    if (S.bus_type[i] != PF_BUS_SLACK) ord_p[i] = np++;
    if (S.bus_type[i] == PF_BUS_PQ) ord_q[i] = nq++;
  }
  Packer pk;
  sable::SymOffsets& so = t->so;
  // level metadata in chunks of whole rows: read in place from the LDS image
  // by LDS-resident slices, staged chunk by chunk in LDS by HBM-resident ones
  sable::LevelChunks chunks;
  // HBM-resident slices of S scenarios: S as large as keeps at least one
  // slice per compute unit and leaves room in LDS for the tail copy (its
  // tail-column blocks, pivot inverses and right-hand sides) and at least
  // 2048 words of staged metadata; the chunk budget takes what remains.
  // S = 1 always fits: the tail holds at most 32 x 32 blocks.
  const int n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  // the LDS copy of the tail: per scenario its tail-column blocks (stride
  // odd, so that the scenarios' copies start in different banks), pivot
  // inverses and right-hand sides, then the tail program's solve prefix
  const size_t tail_nbs = S.tail_cblk.size() | 1;
  auto tail_bytes = [&](int sl) {
    return (size_t)sl * tsz * (4 * tail_nbs + 6 * (size_t)S.tail_t) + 4 * (size_t)S.tail_prog_prefix;
  };
  int hbm_slice = 1;
  while (hbm_slice < sable::kMaxSlice && batch / (2 * hbm_slice) >= n_cu) hbm_slice *= 2;
  while (hbm_slice > 1 && sable::kScratchBytes + tail_bytes(hbm_slice) + 4 * 2048 > max_lds) hbm_slice /= 2;
  if (sable::kScratchBytes + tail_bytes(hbm_slice) + 4 * 2048 > max_lds) {
    delete t;
    return fail(PF_EINVAL, "pf_template_build: the dense tail does not fit in LDS");
  }
  // the slice's right-hand side / solution vector y of the triangular
  // solves lives in LDS too when that leaves the full metadata budget
  const size_t y_bytes = ((size_t)2 * S.nb * hbm_slice * tsz + 15) / 16 * 16;
  size_t room = (max_lds - sable::kScratchBytes - tail_bytes(hbm_slice)) / 4;
  const bool y_in_lds = room >= y_bytes / 4 + kChunkInts;
  if (y_in_lds) room -= y_bytes / 4;
  const int32_t budget = (int32_t)std::min<size_t>(kChunkInts, room / 4 * 4);
  rc = sable::build_level_chunks(S, budget, chunks, err);
  if (rc != 0) { delete t; return fail(PF_EINVAL, err); }
  so.bus_type = (int)pk.add(S.bus_type); so.bus_blk = (int)pk.add(S.bus_blk);
  so.y_rp = (int)pk.add(S.y_rp); so.y_ci = (int)pk.add(S.y_ci);
  so.y_g = (int)pk.add(S.y_g); so.y_b = (int)pk.add(S.y_b);
  so.rp = (int)pk.add(S.rp); so.ci = (int)pk.add(S.ci); so.diag = (int)pk.add(S.diag);
  so.fill4 = (int)pk.add(S.fill4);
  so.tail_pos = (int)pk.add(S.tail_pos); so.tail_split = (int)pk.add(S.tail_split);
  so.tail_mask = (int)pk.add(S.tail_mask);
  so.f_ptr = (int)pk.add(chunks.f_ptr); so.f_blob = (int)pk.add(chunks.f_blob);
  so.fs_ptr = (int)pk.add(chunks.fs_ptr); so.fs_blob = (int)pk.add(chunks.fs_blob);
  so.bs_ptr = (int)pk.add(chunks.bs_ptr); so.bs_blob = (int)pk.add(chunks.bs_blob);
  so.newton_bytes = (int)pk.align();
  so.ut_ptr = (int)pk.add(chunks.ut_ptr); so.ut_blob = (int)pk.add(chunks.ut_blob);
  so.lt_ptr = (int)pk.add(chunks.lt_ptr); so.lt_blob = (int)pk.add(chunks.lt_blob);
  so.tt_ptr = (int)pk.add(chunks.tt_ptr); so.tt_pairs = (int)pk.add(chunks.tt_pairs);
  so.y_tr = (int)pk.add(S.y_tr);
  so.adj_bytes = (int)pk.align();
  so.tail_cblk = (int)pk.add(S.tail_cblk);
  so.tail_prog = (int)pk.add(S.tail_prog);
  so.ord_p = (int)pk.add(ord_p); so.ord_q = (int)pk.add(ord_q);
  so.total_bytes = (int)pk.align();
  sable::Dims& dm = t->dims;
  dm.n_bus = S.n_bus; dm.nb = S.nb; dm.nnzb = S.nnzb(); dm.nj = S.nb + S.n_pq; dm.npq = S.n_pq;
  dm.npvpq = S.nb; dm.nlev_l = S.n_levels_l(); dm.nlev_u = S.n_levels_u();
  dm.nlev_f = S.n_task_levels; dm.nlev_fs = S.n_fs_levels;
  dm.nlev_bs = (int)S.lev_um_ptr.size() - 1;
  dm.tail_t = S.tail_t; dm.tail_base = S.tail_base;
  dm.nch_f = (int)chunks.f_ptr.size() - 1;
  dm.nch_fs = (int)chunks.fs_ptr.size() - 1;
  dm.nch_bs = (int)chunks.bs_ptr.size() - 1;
  // the LDS copy of the tail reads its elimination program from the
  // metadata area (free while the tail is factored) when the area, grown
  // within the room left, holds it
  dm.tail_nbs = (int)tail_nbs;
  dm.tail_prog_ints = (int)S.tail_prog.size();
  dm.tail_prog_prefix = S.tail_prog_prefix;
  const size_t upd_words = S.tail_prog.size() - (size_t)S.tail_prog_prefix;
  dm.tail_prog_lds = upd_words <= room ? 1 : 0;
  dm.chunk_ints = std::max<int>(chunks.max_ints, dm.tail_prog_lds ? (int)(upd_words + 3) / 4 * 4 : 0);
  dm.tail_nblk = (int)S.tail_cblk.size();
  dm.nch_ut = (int)chunks.ut_ptr.size() - 1;
  dm.nch_lt = (int)chunks.lt_ptr.size() - 1;

  // ---- launch shape: LDS-resident slices of S <= 4 scenarios (256 threads,
  // one wavefront per scenario's register-resident tail) when they fit,
  // choosing S to maximise the scenarios resident per CU; HBM-resident
  // slices of up to 16 scenarios otherwise
  t->lay = make_layout(S.n_bus, S.nb, S.nnzb(), 1);
  t->llay = make_lds_layout(S.n_bus, S.nb, S.nnzb(), t->fp32);
  const size_t lds_cu = std::max<size_t>(max_lds, (size_t)prop.maxSharedMemoryPerMultiProcessor);
  const size_t per_scen = 8 * (size_t)t->llay.sd + tsz * (size_t)t->llay.st;
  int best_s = 0;
  size_t best_score = 0;
  const int res_nt = sable::res_newton_threads(t->fp32);
  const bool res_ok = opt.block_threads == 0 || opt.block_threads == res_nt;
  for (int sl : {4, 2, 1}) {
    if (!res_ok || sl > sable::kResMaxSlice) continue;
    const size_t need = sable::kScratchBytes + (size_t)so.newton_bytes + sl * per_scen;
    if (need > max_lds) continue;
    const size_t score = (lds_cu / need) * sl;
    if (score > best_score) { best_score = score; best_s = sl; }
  }
  int nt = opt.block_threads;
  t->wstride = 0;
  t->gmin = 4;
  // the adjoint: LDS-resident slices (256 threads, the tail in registers)
  // whenever the Newton slices are, as wide as fits
  t->alay = make_adj_layout(S.n_bus, S.nb, S.nnzb());
  const size_t per_adj = 8 * (size_t)t->alay.sd + tsz * (size_t)t->alay.st;
  t->adj_slice = 0;
  if (best_s > 0) {
    for (int sl : {4, 2, 1}) {
      const size_t need = sable::kScratchBytes + (size_t)so.adj_bytes + sl * per_adj;
      if (need <= max_lds) { t->adj_slice = sl; t->adj_nt = sable::kResThreads; t->adj_lds = need; break; }
    }
    // no LDS-resident adjoint slice fits: both run HBM-resident, where the
    // adjoint reads the forward solve's slice workspace in place
    if (t->adj_slice == 0) best_s = 0;
  }
  if (best_s > 0) {
    t->lds_res = true;
    t->slice = best_s;
    t->lds_bytes = sable::kScratchBytes + (size_t)so.newton_bytes + best_s * per_scen;
    nt = res_nt;
  } else {
    // HBM-resident: S scenarios interleaved per slice, S as large as keeps
    // at least one slice per compute unit
    t->lds_res = false;
    const int sl = hbm_slice;
    t->slice = sl;
    // grouped per-bus values: a slice of several scenarios reads a bus's
    // values of all of them at once, a slice of one reads them in pairs
    t->lay = make_layout(S.n_bus, S.nb, S.nnzb(), sl > 1 ? 8 : 2);
    t->lds_bytes = sable::kScratchBytes + 4 * (size_t)dm.chunk_ints + tail_bytes(sl);
    t->lds_bytes = (t->lds_bytes + 15) / 16 * 16;
    dm.y_lds_off = 0;
    if (y_in_lds) {
      dm.y_lds_off = (int)t->lds_bytes;
      t->lds_bytes += y_bytes;
    }
    // the adjoint reads this slice workspace in place
    t->adj_slice = -sl;
    t->adj_nt = 1024;   // as the Newton kernel: more lanes per level of the transposed solves
    t->adj_lds = t->lds_bytes;
    // a full workgroup of 16 wavefronts: measured fastest for every slice
    // width (more lanes per level of the elimination schedule)
    if (nt == 0) nt = 1024;
  }
  t->nt = nt;

  he = hipMalloc(&t->d_sym, pk.buf.size());
  if (he != hipSuccess) { delete t; return fail(PF_ENOMEM, "pf_template_build: device allocation (pattern)"); }
  he = hipMemcpy(t->d_sym, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice);
  if (he != hipSuccess) { pf_template_destroy(t); return hip_fail(he, "pf_template_build: upload"); }

  // ---- workspace.  LDS-resident slices and HBM-resident slices of one
  // scenario use the per-scenario layout; wider HBM-resident slices use the
  // slice workspace only (their adjoint reads it in place), and the dense
  // Jacobian export borrows it as per-scenario scratch
  const bool scen_ws = t->lds_res || t->slice == 1;
  const size_t bd = scen_ws ? (size_t)batch * t->lay.sd * 8 : 0,
               bt = scen_ws ? (size_t)batch * t->lay.st * tsz : 0,
               bi = (size_t)batch * 4 * sizeof(int);
  if ((scen_ws && (hipMalloc(&t->ws_d, bd) != hipSuccess || hipMalloc(&t->ws_t, bt) != hipSuccess)) ||
      hipMalloc(&t->ws_i, bi) != hipSuccess) {
    pf_template_destroy(t);
    return fail(PF_ENOMEM, "pf_template_build: device allocation (workspace)");
  }
  size_t bsl = 0;
  if (!t->lds_res && t->slice > 1) {
    const size_t slices = (size_t)(batch + t->slice - 1) / t->slice;
    const size_t sd = slices * t->slice * t->lay.sd * 8, stt = slices * t->slice * t->lay.st * tsz;
    if (hipMalloc(&t->wsl_d, sd) != hipSuccess || hipMalloc(&t->wsl_t, stt) != hipSuccess) {
      pf_template_destroy(t);
      return fail(PF_ENOMEM, "pf_template_build: device allocation (slice workspace)");
    }
    bsl = sd + stt;
  }
  he = hipMemset(t->ws_i, 0xff, bi);
  if (he == hipSuccess && std::max(t->lds_bytes, t->adj_lds) > 64 * 1024)
    he = sable::set_lds_limits(std::max(t->lds_bytes, t->adj_lds));
  if (he == hipSuccess) he = hipDeviceSynchronize();
  if (he != hipSuccess) { pf_template_destroy(t); return hip_fail(he, "pf_template_build: set-up"); }
  t->ws_bytes = pk.buf.size() + bd + bt + bi + bsl;
  rc = build_operator_tables(t);
  if (rc != PF_OK) {
    const std::string msg = g_err;
    pf_template_destroy(t);
    return fail(rc, msg);
  }
  *out = t;
  return PF_OK;
}

int pf_template_info(const pf_template* t, pf_template_stats* out) {
  g_err.clear();
  if (!t || !out) return fail(PF_EINVAL, "pf_template_info: NULL argument");
  fill_stats(t->sym, out);
  out->workspace_bytes = t->ws_bytes;
  out->batch = t->batch;
  out->lds_resident = t->lds_res ? 1 : 0;
  out->block_threads = t->nt;
  out->lds_bytes = (int32_t)t->lds_bytes;
  out->slice_width = t->slice;
  return PF_OK;
}

int pf_template_destroy(pf_template* t) {
  g_err.clear();
  if (!t) return PF_OK;
  DeviceGuard g(t->device);
  (void)hipDeviceSynchronize();
  if (t->d_sym) (void)hipFree(t->d_sym);
  if (t->ws_d) (void)hipFree(t->ws_d);
  if (t->ws_t) (void)hipFree(t->ws_t);
  if (t->ws_i) (void)hipFree(t->ws_i);
  if (t->wsl_d) (void)hipFree(t->wsl_d);
  if (t->wsl_t) (void)hipFree(t->wsl_t);
  if (t->d_ops) (void)hipFree(t->d_ops);
  if (t->d_opef) (void)hipFree(t->d_opef);
  delete t;
  return PF_OK;
}

int pf_solve_batch(pf_template* t, const double* pd, const double* qd, const double* pg,
                   const double* vset, double* vm, double* va, int32_t* iters, int32_t* status,
                   double* final_mismatch, void* hip_stream) {
  g_err.clear();
  if (!t) return fail(PF_EINVAL, "pf_solve_batch: template is NULL");
  if (!pd || !qd || !vset || !vm || !va) return fail(PF_EINVAL, "pf_solve_batch: NULL input/output array");
  DeviceGuard g(t->device);
  sable::KParams kp = base_params(t);
  kp.mode = sable::MODE_SOLVE;
  kp.pd = pd; kp.qd = qd; kp.pg = pg; kp.vset = vset;
  kp.vm_out = vm; kp.va_out = va;
  kp.iters_out = iters; kp.status_out = status; kp.fnorm_out = final_mismatch;
  const int grid = (t->batch + t->slice - 1) / t->slice;
  hipError_t he = sable::launch_newton(kp, t->fp32, t->slice, grid, t->nt, t->lds_bytes, t->lds_res,
                                       static_cast<hipStream_t>(hip_stream));
  if (he != hipSuccess) return hip_fail(he, "pf_solve_batch: launch");
  t->have_factors = t->opt.keep_factors != 0;
  return PF_OK;
}


int pf_adjoint_batch(pf_template* t, const double* g_vm, const double* g_va, double* g_pd,
                     double* g_qd, double* g_pg, double* g_vset, void* hip_stream) {
  return adjoint_impl("pf_adjoint_batch", t, g_vm, g_va, nullptr, nullptr, g_pd, g_qd, g_pg, g_vset,
                      hip_stream);
}

int pf_adjoint_completed_batch(pf_template* t, const double* g_vm, const double* g_va,
                               const double* g_pg_out, const double* g_qg_out, double* g_pd,
                               double* g_qd, double* g_pg, double* g_vset, void* hip_stream) {
  return adjoint_impl("pf_adjoint_completed_batch", t, g_vm, g_va, g_pg_out, g_qg_out, g_pd, g_qd, g_pg,
                      g_vset, hip_stream);
}

int pf_recover_batch(pf_template* t, const double* pd, const double* qd, const double* pg,
                     const double* vm, const double* va, double* pg_out, double* qg_out,
                     void* hip_stream) {
  g_err.clear();
  if (!t) return fail(PF_EINVAL, "pf_recover_batch: template is NULL");
  if (!pd || !qd || !vm || !va) return fail(PF_EINVAL, "pf_recover_batch: NULL input");
  DeviceGuard g(t->device);
  sable::KParams kp = base_params(t);
  kp.pd = pd; kp.qd = qd; kp.pg = pg; kp.vm_in = vm; kp.va_in = va;
  kp.pg_out = pg_out; kp.qg_out = qg_out;
  hipError_t he = sable::launch_recover(kp, static_cast<hipStream_t>(hip_stream));
  if (he != hipSuccess) return hip_fail(he, "pf_recover_batch: launch");
  return PF_OK;
}

int pf_eval_batch(pf_template* t, int32_t mode, int32_t count, const double* pd, const double* qd,
                  const double* pg, const double* vset, const double* vm, const double* va,
                  const double* rhs, double* out, void* hip_stream) {
  g_err.clear();
  if (!t) return fail(PF_EINVAL, "pf_eval_batch: template is NULL");
  if (count <= 0 || count > t->batch) return fail(PF_EINVAL, "pf_eval_batch: count out of range");
  if (!pd || !qd || !vset || !vm || !va || !out) return fail(PF_EINVAL, "pf_eval_batch: NULL array");
  if (mode == PF_EVAL_ADJOINT && !rhs) return fail(PF_EINVAL, "pf_eval_batch: rhs is NULL");
  DeviceGuard g(t->device);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  sable::KParams kp = base_params(t);
  kp.pd = pd; kp.qd = qd; kp.pg = pg; kp.vset = vset; kp.vm_in = vm; kp.va_in = va;
  kp.rhs = rhs; kp.out = out; kp.count = count;
  t->have_factors = false;   // the evaluation reuses the workspace
  hipError_t he;
  const int grid = (count + t->slice - 1) / t->slice;
  switch (mode) {
    case PF_EVAL_MISMATCH:
      kp.mode = sable::MODE_EVAL_MISMATCH;
      he = sable::launch_newton(kp, t->fp32, t->slice, grid, t->nt, t->lds_bytes, t->lds_res, st);
      break;
    case PF_EVAL_STEP:
      kp.mode = sable::MODE_EVAL_STEP;
      he = sable::launch_newton(kp, t->fp32, t->slice, grid, t->nt, t->lds_bytes, t->lds_res, st);
      break;
    case PF_EVAL_JACOBIAN:
      he = sable::launch_jacobian_dense(kp, count, st);
      break;
    case PF_EVAL_FILL:
      kp.mode = sable::MODE_EVAL_FILL;
      he = sable::launch_newton(kp, t->fp32, t->slice, grid, t->nt, t->lds_bytes, t->lds_res, st);
      break;
    case PF_EVAL_ADJOINT:
      kp.mode = sable::MODE_EVAL_FACTOR;
      he = sable::launch_newton(kp, t->fp32, t->slice, grid, t->nt, t->lds_bytes, t->lds_res, st);
      if (he == hipSuccess) {
        kp.mode = sable::MODE_EVAL_ADJOINT;
        const int aw = t->adj_slice < 0 ? -t->adj_slice : t->adj_slice;
        he = sable::launch_adjoint(kp, t->fp32, t->adj_slice, aw ? (count + aw - 1) / aw : count,
                                   aw ? t->adj_nt : t->nt, t->adj_lds, st);
      }
      break;
    default:
      return fail(PF_EINVAL, "pf_eval_batch: unknown mode");
  }
  if (he != hipSuccess) return hip_fail(he, "pf_eval_batch: launch");
  return PF_OK;
}

int pf_operator_pattern(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
                        const int32_t* y_indices, int32_t which, int32_t* n_rows, int32_t* n_cols,
                        int32_t* nnz, int32_t* nnz_base, int32_t* indptr, int32_t* indices, int32_t* pos) {
  g_err.clear();
  if (n_bus < 2 || !bus_type || !y_indptr || !y_indices)
    return fail(PF_EINVAL, "pf_operator_pattern: bad network arrays");
  if (which < 0 || which >= sable::OP_COUNT) return fail(PF_EINVAL, "pf_operator_pattern: unknown operator");
  const int32_t nnzY = y_indptr[n_bus];
  if (y_indptr[0] != 0 || nnzY < 0) return fail(PF_EINVAL, "pf_operator_pattern: bad y_indptr");
  for (int32_t i = 0; i < n_bus; ++i)
    if (y_indptr[i + 1] < y_indptr[i]) return fail(PF_EINVAL, "pf_operator_pattern: bad y_indptr");
  // the template stores Y_bus with each row's columns sorted; do the same
  std::vector<int32_t> ci(y_indices, y_indices + nnzY);
  for (int32_t i = 0; i < n_bus; ++i) std::sort(ci.begin() + y_indptr[i], ci.begin() + y_indptr[i + 1]);
  sable::OperatorSet ops;
  std::string err;
  const int rc = sable::build_operators(n_bus, bus_type, y_indptr, ci.data(), ops, err);
  if (rc != PF_OK) return fail(rc, "pf_operator_pattern: " + err);
  const sable::OperatorPattern& op = ops.op[which];
  if (n_rows) *n_rows = op.rows;
  if (n_cols) *n_cols = op.cols;
  if (nnz) *nnz = (int32_t)op.indices.size();
  if (nnz_base) *nnz_base = (int32_t)ops.base.size();
  if (indptr) std::copy(op.indptr.begin(), op.indptr.end(), indptr);
  if (indices) std::copy(op.indices.begin(), op.indices.end(), indices);
  if (pos) std::copy(op.pos.begin(), op.pos.end(), pos);
  return PF_OK;
}

int pf_operator_values(pf_template* t, int32_t which, int32_t count, const double* vm, const double* va,
                       double* values, void* hip_stream) {
  sable::OpParams p{};
  int dev = 0;
  int rc = sable::operator_params(t, which, count, vm, va, values, "pf_operator_values", p, dev);
  if (rc != PF_OK) return rc;
  DeviceGuard g(dev);
  if ((size_t)count > t->opef_count) {   // grow the state buffer (previous work may still read it)
    (void)hipDeviceSynchronize();
    if (t->d_opef) (void)hipFree(t->d_opef);
    t->d_opef = nullptr;
    t->opef_count = 0;
    hipError_t he = hipMalloc(&t->d_opef, (size_t)count * t->sym.n_bus * 4 * sizeof(double));
    if (he != hipSuccess) {
      t->d_opef = nullptr;
      return fail(PF_ENOMEM, "pf_operator_values: device allocation (per-bus state)");
    }
    t->opef_count = (size_t)count;
  }
  p.ef = t->d_opef;
  hipError_t he = sable::launch_operator_values(p, static_cast<hipStream_t>(hip_stream));
  if (he != hipSuccess) return hip_fail(he, "pf_operator_values: launch");
  return PF_OK;
}

int pf_operator_bde_csr(pf_template* t, int32_t which, int32_t count, int64_t* crow, int64_t* col,
                        void* hip_stream) {
  g_err.clear();
  if (!t) return fail(PF_EINVAL, "pf_operator_bde_csr: template is NULL");
  if (which < 0 || which >= sable::OP_COUNT) return fail(PF_EINVAL, "pf_operator_bde_csr: unknown operator");
  if (count < 0) return fail(PF_EINVAL, "pf_operator_bde_csr: negative count");
  if (!crow || (count > 0 && t->op_nnz[which] > 0 && !col))
    return fail(PF_EINVAL, "pf_operator_bde_csr: NULL output array");
  DeviceGuard g(t->device);
  const int32_t* d = static_cast<const int32_t*>(t->d_ops);
  hipError_t he = sable::launch_bde_csr(d + t->op_ip_off[which], d + t->op_ix_off[which], t->op_rows[which],
                                        t->op_cols[which], t->op_nnz[which], count, crow, col,
                                        static_cast<hipStream_t>(hip_stream));
  if (he != hipSuccess) return hip_fail(he, "pf_operator_bde_csr: launch");
  return PF_OK;
}

int pf_debug_phase_clocks(uint64_t* ticks, int32_t n, int32_t reset, double* ticks_per_second) {
  g_err.clear();
  if (n < 0 || (n > 0 && !ticks)) return fail(PF_EINVAL, "pf_debug_phase_clocks: bad buffer");
  std::vector<unsigned long long> buf(std::max(n, 1), 0ull);
  hipError_t he = sable::read_phase_clocks(buf.data(), n, reset != 0);
  if (he == hipErrorNotSupported)
    return fail(PF_EINVAL, "pf_debug_phase_clocks: library built without per-phase clocks");
  if (he != hipSuccess) return hip_fail(he, "pf_debug_phase_clocks");
  for (int32_t i = 0; i < n; ++i) ticks[i] = buf[i];
  if (ticks_per_second) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      return fail(PF_EHIP, "pf_debug_phase_clocks: wall-clock rate query");
    *ticks_per_second = 1e3 * (double)khz;
  }
  return PF_OK;
}

int pf_template_block_pattern(const pf_template* t, int32_t* row_bus, int32_t* col_bus) {
  g_err.clear();
  if (!t || !row_bus || !col_bus) return fail(PF_EINVAL, "pf_template_block_pattern: NULL argument");
  const sable::Symbolic& S = t->sym;
  for (int32_t p = 0; p < S.nnzb(); ++p) {
    row_bus[p] = S.blk_bus[S.prow[p]];
    col_bus[p] = S.blk_bus[S.ci[p]];
  }
  return PF_OK;
}

}  // extern "C"
