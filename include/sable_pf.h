/*
 * sable_pf.h -- C ABI of the batched Newton-Raphson AC power-flow library
 * for AMD Instinct MI355X (gfx950).
 *
 * Problem (paper: "SABLE: GPU-Based Power Flow Accelerator for Sparsity-Aware
 * Batched Learning"):
 *   Buses are split into PQ (load) buses D, PV (generator) buses G and one
 *   slack bus R (Sec. II-A).  All scenarios of a batch share Y_bus = G + jB
 *   and the bus types; scenario b brings loads p_d, q_d, PV dispatch p_g and
 *   |V| setpoints on G u R (the decision block x, eq. ynn).  For each scenario
 *   the library solves the step-1 completion F1(z1) = 0 with
 *   z1 = (|V| on D, theta on B\R), F1 = (dP on B\R, dQ on D),
 *   dP = P_spec - P, dQ = Q_spec - Q, P_spec = p_g - p_d, Q_spec = q_g - q_d
 *   and S = P + jQ = V o conj(Y_bus V), by full Newton-Raphson from the flat
 *   start (eqs. reduced_pf_system, nr_linear_system_completion,
 *   step1_jacobian; flat start and tolerance of Sec. IV-A), and returns the
 *   implicit-differentiation gradients of a loss (J1^T lambda = g_z1 and the
 *   J3 term, backward pass of Sec. II-B).
 *
 * Units: per-unit powers and voltages, angles in radians, slack angle 0.
 *
 * Return codes (every function): PF_OK = 0, or a negative PF_E* code; the
 * matching human-readable message is available from pf_last_error() (per
 * thread).  Per-scenario numerical outcomes are NOT call errors: they are
 * written to status[b] (PF_STATUS_*).
 *
 * Memory: network arrays passed to pf_template_build / pf_ybus_from_branches
 * are host arrays, copied by the call; batch arrays passed to pf_solve_batch
 * / pf_adjoint_batch are caller-owned DEVICE arrays (contiguous, row-major
 * [batch][n_bus] float64 unless stated), never freed or retained by the
 * library.  A template owns all its device workspace, allocated once in
 * pf_template_build and released by pf_template_destroy.
 *
 * Streams: pf_solve_batch and pf_adjoint_batch enqueue work on the given HIP
 * stream (hipStream_t passed as void*, NULL = default stream) and return
 * without synchronising.  pf_template_build and pf_template_destroy are
 * synchronous.  A template is not thread-safe; distinct templates are
 * independent.
 */
#ifndef SABLE_PF_H
#define SABLE_PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define PF_OK 0
#define PF_EINVAL (-1)     /* bad size, pointer, option or bus type */
#define PF_ETOPOLOGY (-2)  /* not exactly one slack, isolated bus, disconnected network */
#define PF_ENOMEM (-3)     /* device or host allocation failed */
#define PF_EHIP (-4)       /* HIP runtime error (launch, copy, no device) */
#define PF_ESTATE (-5)     /* adjoint without a preceding solve that kept its factors */

/* bus types */
#define PF_BUS_PQ 0
#define PF_BUS_PV 1
#define PF_BUS_SLACK 2

/* precision policy (stagewise mixed precision, Sec. III-C, Table I) */
#define PF_FP64 0   /* Jacobian, LU factors and triangular solves in FP64 */
#define PF_MIXED 1  /* LU factors and triangular solves in FP32; mismatch, convergence
                       test, Jacobian evaluation, state update and the refinement
                       residual in FP64 */

/* per-scenario outcome written to status[b] */
#define PF_STATUS_CONVERGED 0   /* ||F1||_inf < tol */
#define PF_STATUS_MAX_ITER 1    /* still >= tol after max_iter updates */
#define PF_STATUS_NON_FINITE 2  /* mismatch became NaN or Inf */
#define PF_STATUS_ZERO_PIVOT 3  /* a 2x2 pivot block is numerically singular: one of its two
                                   scalar pivots is <= eps * |row of the block| (eps = 1e-14
                                   for FP64 factors, 1e-7 for FP32) or its inverse is not finite */

typedef struct pf_template pf_template; /* opaque */

typedef struct {
  double tol;            /* Newton stops when ||F1||_inf < tol (pu); default 1e-8 */
  int32_t max_iter;      /* maximum Newton updates; default 20; 0 = only evaluate */
  int32_t precision;     /* PF_FP64 (default) or PF_MIXED */
  int32_t refine_steps;  /* PF_MIXED: FP64-residual refinement solves per Newton step;
                            default 2; ignored for PF_FP64 */
  int32_t keep_factors;  /* 1 (default): after convergence re-evaluate J1 and refactor
                            at the solution and keep the factors for pf_adjoint_batch */
  int32_t block_threads; /* threads per workgroup, 0 = automatic (64..1024); LDS-resident
                            slices always run 512 threads, so any other nonzero value
                            selects HBM-resident slices */
  int32_t refine_adaptive; /* PF_MIXED forward solve: 0 (default) applies all refine_steps
                            refinement solves; 1 computes the FP64 residual r of the
                            current correction and refines only while
                            ||r||_inf > max(min(0.1, ||F1||_inf) ||F1||_inf, 0.1 tol)
                            (an inexact-Newton forcing term that keeps the convergence
                            quadratic), at most refine_steps times.  The convergence test
                            is always on the FP64 mismatch, so the final accuracy is the
                            same; the adjoint always applies refine_steps steps */
} pf_options;

typedef struct {
  int32_t n_bus, n_pv, n_pq;
  int32_t n_j;             /* Newton unknowns: (n_bus - 1) + n_pq */
  int32_t nnz_ybus;
  int64_t nnz_j1;          /* scalar nonzeros of J1 */
  int32_t n_blocks;        /* 2x2 block rows (non-slack buses) */
  int32_t nnzb_lu;         /* 2x2 blocks of L+U including the diagonal */
  int64_t nnz_lu;          /* scalar nonzeros of L+U over the real unknowns */
  int64_t n_block_updates; /* block multiply-subtracts per factorisation */
  int32_t n_levels_l;      /* level sets of the factorisation / forward solve */
  int32_t n_levels_u;      /* level sets of the backward solve */
  int32_t max_row_blocks;
  double fill_ratio;       /* nnz_lu / nnz_j1 */
  double factor_flops;     /* flops of one factorisation (2x2 block arithmetic) */
  size_t workspace_bytes;  /* device bytes owned by the template */
  int32_t batch;
  int32_t lds_resident;    /* 1: factors and state of a scenario live in LDS */
  int32_t block_threads;   /* threads per workgroup used by the solve kernels */
  int32_t lds_bytes;       /* dynamic LDS per workgroup */
  int32_t slice_width;     /* scenarios per workgroup of the Newton kernel */
} pf_template_stats;

/* Fills *opt with the defaults listed above.  Never fails. */
void pf_default_options(pf_options* opt);

/* Message of the last failing call on this thread ("" if none).  Owned by
   the library, valid until the next call on the same thread. */
const char* pf_last_error(void);

/*
 * Assemble Y_bus (CSR, sorted columns, every diagonal present) from a
 * pi-model branch list: series admittance 1/(r + jx) between the ends and
 * half of the total line charging bc at each end; no taps or shunts (the
 * paper takes Y_bus as given, Sec. II-A).  Host arrays.  indptr has n_bus+1
 * entries; indices/g/b have `capacity` entries.  *nnz_out receives the
 * number of nonzeros; if it exceeds capacity, PF_EINVAL is returned and only
 * *nnz_out is written (call again with enough room).
 */
int pf_ybus_from_branches(int32_t n_bus, int32_t n_branch, const int32_t* from, const int32_t* to,
                          const double* r, const double* x, const double* b_charging,
                          int32_t* indptr, int32_t* indices, double* g, double* b,
                          int32_t capacity, int32_t* nnz_out);

/*
 * One-time symbolic analysis + device set-up for a network and a batch size
 * (one-time symbolic analysis, Sec. III-B; the fixed template of the
 * block-diagonal embedding, eq. BDE_global, is kept as ONE per-scenario
 * pattern shared by the batch).  Host inputs: bus_type[n_bus] (PF_BUS_*),
 * Y_bus in CSR (y_indptr[n_bus+1], y_indices/y_g/y_b[y_indptr[n_bus]],
 * int32 indices, columns in any order, no duplicates).  opt may be NULL
 * (defaults).  Requires a HIP device; allocates all workspace for `batch`
 * scenarios.  On success *out receives the template.
 * Errors: PF_EINVAL, PF_ETOPOLOGY, PF_ENOMEM, PF_EHIP.
 */
int pf_template_build(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
                      const int32_t* y_indices, const double* y_g, const double* y_b,
                      int32_t batch, const pf_options* opt, pf_template** out);

/* Sizes of the analysis.  Host-only, never touches the device. */
int pf_template_info(const pf_template* tpl, pf_template_stats* out);

/* The 2x2-block pattern of L+U in the library's storage order (one-time
   symbolic analysis, Sec. III-B): host outputs row_bus[nnzb_lu] and
   col_bus[nnzb_lu], the buses of each block's row and column.  Host-only.
   Errors: PF_EINVAL. */
int pf_template_block_pattern(const pf_template* tpl, int32_t* row_bus, int32_t* col_bus);

/* Releases the template and its device memory (synchronises the device).
   NULL is accepted. */
int pf_template_destroy(pf_template* tpl);

/*
 * Host-only symbolic analysis (no device needed): fills the pattern
 * statistics of *out (workspace_bytes, lds_* and block_threads are 0) and,
 * if bus_order is not NULL, the elimination order of the non-slack buses
 * (bus_order[n_bus - 1]).  For tests and capacity planning.
 */
int pf_symbolic_analyze(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
                        const int32_t* y_indices, pf_template_stats* out, int32_t* bus_order);

/*
 * Batched Newton-Raphson solve (Step 1, Sec. II-B) of `batch` scenarios
 * (the value given at build) from the flat start.  Device inputs
 * [batch][n_bus]: pd, qd (loads; read on non-slack buses), pg (dispatch, read
 * on PV buses only; NULL = zero), vset (|V| setpoints, read on PV and slack
 * buses).  Device outputs: vm, va [batch][n_bus] (the completed voltage
 * magnitudes and angles, slack angle 0), iters[batch] (updates applied),
 * status[batch] (PF_STATUS_*), final_mismatch[batch] (||F1||_inf at the
 * returned state; NaN if non-finite).  Any output pointer except vm/va may be
 * NULL.  Converged scenarios stop updating while the others continue.  With
 * keep_factors the converged state and the LU factors of J1 at it are kept
 * for pf_adjoint_batch.
 * Errors: PF_EINVAL (NULL template/inputs), PF_EHIP (launch failure).
 */
int pf_solve_batch(pf_template* tpl, const double* pd, const double* qd, const double* pg,
                   const double* vset, double* vm, double* va, int32_t* iters, int32_t* status,
                   double* final_mismatch, void* hip_stream);

/*
 * Adjoint of the most recent pf_solve_batch on this template (backward pass
 * of Sec. II-B).  Device inputs g_vm, g_va [batch][n_bus]: dL/d|V| and
 * dL/dtheta at the returned solution.  Solves J1^T lambda = g_z1 with the
 * kept LU factors (U^T then L^T; PF_MIXED adds refine_steps FP64-residual
 * refinement steps) and writes device outputs [batch][n_bus]:
 *   g_pd   = dL/dp_d   (+lambda_P on non-slack buses, 0 on the slack)
 *   g_qd   = dL/dq_d   (+lambda_Q on PQ buses, 0 elsewhere)
 *   g_pg   = dL/dp_g   (-lambda_P on PV buses, 0 elsewhere)
 *   g_vset = dL/dV_set (g_vm - (J3^T lambda) on PV and slack buses, 0 elsewhere)
 * Any output may be NULL.  Scenarios whose solve did not converge get zero
 * gradients.  Errors: PF_EINVAL, PF_ESTATE (no solve yet, or keep_factors=0),
 * PF_EHIP.
 */
int pf_adjoint_batch(pf_template* tpl, const double* g_vm, const double* g_va, double* g_pd,
                     double* g_qd, double* g_pg, double* g_vset, void* hip_stream);

/*
 * Step 2 of the forward completion (eq. F2_completion): the generation block
 * of the completed PF buffer y (eq. y_and_F_base) at a solution (vm, va).
 * The equality rows left out of F1 (dP on the slack bus, dQ on PV and slack
 * buses) are zero at the solution and contain z2 = (p_g on the slack bus,
 * q_g on PV and slack buses) with unit coefficients, so with
 * S = P + jQ = V o conj(Y_bus V) evaluated in FP64:
 *   pg_out = P + pd on the slack bus, pg (x, passed through) on PV buses,
 *            0 on PQ buses
 *   qg_out = Q + qd on PV and slack buses, 0 on PQ buses
 * Device inputs [batch][n_bus]: pd, qd, pg (NULL = zero), vm, va (normally
 * what pf_solve_batch returned; any state is accepted and every scenario is
 * evaluated, whatever its solve status).  Device outputs [batch][n_bus]:
 * pg_out, qg_out (either may be NULL).  Reads only the template's pattern,
 * not its workspace, so it may run before or after any solve.  Asynchronous
 * on hip_stream.  Errors: PF_EINVAL (NULL template or input), PF_EHIP.
 */
int pf_recover_batch(pf_template* tpl, const double* pd, const double* qd, const double* pg,
                     const double* vm, const double* va, double* pg_out, double* qg_out,
                     void* hip_stream);

/*
 * Adjoint of the full two-step completion (chain-rule equation and the J2
 * and vbar2 equations of the backward pass, Sec. II-B): as pf_adjoint_batch,
 * for a loss that also depends on the recovered generation.  Extra device
 * inputs [batch][n_bus]: g_pg_out = dL/d(pg_out), read on slack and PV
 * buses, and g_qg_out = dL/d(qg_out), read on PV and slack buses; either may
 * be NULL (zero).  The kernel forms vbar2 = -J2^T dL/dz2 with
 * J2 = dF2/d(|V|, theta) (eq. Jstep2_impl) as a transposed product through
 * Y_bus at the kept state, adds it to g_z1 before the J1^T solve and to the
 * |V| entries of g_x after it.  Outputs [batch][n_bus] (any may be NULL):
 *   g_pd   = +lambda_P on non-slack buses; g_pg_out on the slack bus
 *   g_qd   = +lambda_Q on PQ buses; g_qg_out on PV and slack buses
 *   g_pg   = g_pg_out - lambda_P on PV buses, 0 elsewhere
 *   g_vset = g_vm + vbar2 - (J3^T lambda) on PV and slack buses, 0 elsewhere
 * (the load terms on the generator rows are the unit dependence of z2 on the
 * load of its own row).  Scenarios whose solve did not converge get zero
 * gradients.  Errors: PF_EINVAL, PF_ESTATE (no solve yet, or
 * keep_factors=0), PF_EHIP.
 */
int pf_adjoint_completed_batch(pf_template* tpl, const double* g_vm, const double* g_va,
                               const double* g_pg_out, const double* g_qg_out, double* g_pd,
                               double* g_qd, double* g_pg, double* g_vset, void* hip_stream);

/*
 * The base Jacobian template and the operators the layer uses, as sparse
 * matrices for interop (eq. J_base_block; step1_jacobian, Jstep2_impl and
 * Jstep3_impl; block-aware indexing of Sec. III-B).  Orderings, each block
 * ascending by bus: y = (p_g on B\D, q_g on B\D, |V| of every bus, theta of
 * every bus), F = (dP of every bus, dQ of every bus).
 *   PF_OP_BASE: J = dF/dy, 2 n_bus x (2 n_gen + 2 n_bus), n_gen = |B\D|;
 *               dP_i/dp_g,i = dQ_i/dq_g,i = 1 (selectors), voltage blocks on
 *               the Y_bus pattern (diagonal always present)
 *   PF_OP_J1:   J1 = dF1/dz1, rows (dP on B\R, dQ on D), columns
 *               (|V| on D, theta on B\R)
 *   PF_OP_J1T:  J1^T
 *   PF_OP_J2T:  J2^T, J2 = dF2/d(|V|, theta): rows (dP on R, dQ on B\D),
 *               columns (|V| of every bus, theta of every bus)
 *   PF_OP_J3T:  J3^T, J3 = dF1/d|V| on B\D
 * One scenario's pattern is built once; the batch-global operator is the
 * block-diagonal embedding of that pattern (eq. BDE_global: scenario b's block
 * at row offset b*n_rows and column offset b*n_cols), whose CSR value array is
 * exactly values[count][nnz] below (pf_operator_bde_csr writes its row
 * pointers and column indices).
 */
#define PF_OP_BASE 0
#define PF_OP_J1 1
#define PF_OP_J1T 2
#define PF_OP_J2T 3
#define PF_OP_J3T 4

/*
 * CSR pattern of operator `which` for one scenario, from the network alone
 * (host; no device needed).  Host inputs as for pf_template_build (Y_bus rows
 * need not be sorted).  Always writes *n_rows, *n_cols, *nnz and *nnz_base
 * (non-zeros of the base J) when non-NULL; writes indptr[n_rows + 1],
 * indices[nnz] (columns sorted within a row) and pos[nnz_base] (for each
 * base entry, in the base's value order, its position in this operator's
 * value array, or -1 if the operator does not use it: the position map of
 * Algorithm 2) when those pointers are non-NULL, so a first call with NULL
 * arrays queries the sizes.  Errors: PF_EINVAL.
 */
int pf_operator_pattern(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
                        const int32_t* y_indices, int32_t which, int32_t* n_rows, int32_t* n_cols,
                        int32_t* nnz, int32_t* nnz_base, int32_t* indptr, int32_t* indices,
                        int32_t* pos);

/*
 * Values of operator `which` for scenarios [0, count) at the states
 * (vm, va) (device [count][n_bus], FP64): device output values[count][nnz],
 * in the order of pf_operator_pattern's CSR, evaluated in FP64 (Algorithm 1's
 * entry formulas; selectors are 1).  count may exceed the template's batch:
 * only the template's pattern is used, not its workspace.  The operator
 * tables are built with the template; the first call allocates a buffer of
 * 32 * count * n_bus bytes for the per-bus voltages and injections (device
 * memory, released by pf_template_destroy); a later call with a larger count
 * grows that buffer (after a device synchronisation), any other call
 * allocates nothing.  Calls on one template share the buffer: calls that
 * overlap on different streams race.  Asynchronous on hip_stream.
 * Errors: PF_EINVAL, PF_ENOMEM, PF_EHIP.
 */
int pf_operator_values(pf_template* tpl, int32_t which, int32_t count, const double* vm,
                       const double* va, double* values, void* hip_stream);

/*
 * pf_operator_values for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same arguments, values and errors, but the per-bus voltages and
 * injections live in a fixed 32 MiB device array that the library holds on
 * each device it runs on until the process ends, so the call allocates
 * nothing, not even on its first use.  A batch whose state (32 bytes per bus
 * and scenario) exceeds the array is processed in consecutive pieces on
 * hip_stream; a network of more than 2^20 buses is rejected with PF_EINVAL.
 * All calls on one device share the array: calls that overlap on one device
 * (different streams or threads) race.  Asynchronous on hip_stream.
 * Errors: PF_EINVAL, PF_EHIP.
 */
int pf_operator_values_static(pf_template* tpl, int32_t which, int32_t count, const double* vm,
                              const double* va, double* values, void* hip_stream);

/*
 * Row pointers and column indices of the batch-global operator `which` for
 * `count` scenarios: the block-diagonal embedding of one scenario's pattern
 * (eq. BDE_global; scenario b's block at row offset b * n_rows and column
 * offset b * n_cols of pf_operator_pattern, its values at offset b * nnz, so
 * values[count][nnz] of pf_operator_values is this CSR's value array).
 * Device outputs, int64: crow[count * n_rows + 1], col[count * nnz]
 * (caller-owned).  count = 0 writes crow[0] = 0 only.  Asynchronous on
 * hip_stream; allocates nothing.  Errors: PF_EINVAL, PF_EHIP.
 */
int pf_operator_bde_csr(pf_template* tpl, int32_t which, int32_t count, int64_t* crow, int64_t* col,
                        void* hip_stream);

/*
 * Evaluation entry points at a GIVEN state (vm, va device [batch][n_bus]),
 * for kernel-level checks and interop, in the paper's ordering: rows
 * (dP on B\R ascending bus, then dQ on D ascending bus), unknowns
 * (|V| on D ascending, then theta on B\R ascending) (eqs. reduced_pf_system,
 * step1_jacobian).  Scenarios [0, count) are evaluated, count <= batch.
 *   PF_EVAL_MISMATCH: out[count][n_j]        = F1
 *   PF_EVAL_JACOBIAN: out[count][n_j][n_j]   = J1 (dense)
 *   PF_EVAL_STEP:     out[count][n_j]        = dz solving J1 dz = -F1 with the
 *                                              library's LU in the template's
 *                                              precision (+ refinement if mixed)
 *   PF_EVAL_ADJOINT:  out[count][n_j]        = lambda solving J1^T lambda = rhs,
 *                     rhs[count][n_j] given in the unknown ordering
 *   PF_EVAL_FILL:     out[count][4 nnzb_lu]  = the values the Jacobian value
 *                     update (Algorithm 1) writes into the LU positions before
 *                     the factorisation, in the library's block order
 *                     (pf_template_block_pattern), each 2x2 block row-major
 *                     with rows (dP_i, dQ_i) and columns (theta_j, |V|_j) of
 *                     its bus pair; a PV bus's dQ row and |V| column are
 *                     padding (zero, with 1 on its diagonal block's |V|
 *                     entry), fill-in blocks are zero; converted from the
 *                     factor precision to FP64
 * pd/qd/pg/vset as for pf_solve_batch (the Jacobian and the adjoint solve do
 * not read them but they must be valid).  rhs is only read by
 * PF_EVAL_ADJOINT (may be NULL otherwise).
 */
#define PF_EVAL_MISMATCH 0
#define PF_EVAL_JACOBIAN 1
#define PF_EVAL_STEP 2
#define PF_EVAL_ADJOINT 3
#define PF_EVAL_FILL 4
int pf_eval_batch(pf_template* tpl, int32_t mode, int32_t count, const double* pd,
                  const double* qd, const double* pg, const double* vset, const double* vm,
                  const double* va, const double* rhs, double* out, void* hip_stream);

/*
 * Measurement aid: per-phase wall-clock counters of the Newton kernel,
 * present only in the library variant built with -DSABLE_PHASE_CLOCKS
 * (libsablepf_phases.so); the production library returns PF_EINVAL.
 * Workgroup 0 of every Newton launch adds the ticks of the constant-rate wall
 * clock spent in each phase (slots 0..14: set-up, mismatch, fill, factor
 * levels, factor tail, backward tail, backward levels, refinement dV,
 * refinement residual, refinement forward levels, refinement tail,
 * refinement backward levels, other, kept-factor refresh, outputs) and event
 * counts (slot 16: launches, 17: Newton corrections, 18: refinement steps).
 * Copies the first n slots to the host array ticks[n] after a device
 * synchronisation, clears them when reset != 0, and writes the clock rate
 * to *ticks_per_second when not NULL.  Errors: PF_EINVAL, PF_EHIP.
 */
int pf_debug_phase_clocks(uint64_t* ticks, int32_t n, int32_t reset, double* ticks_per_second);

#ifdef __cplusplus
}
#endif

#endif /* SABLE_PF_H */
