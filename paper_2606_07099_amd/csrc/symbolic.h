// One-time symbolic analysis for the batched Newton power flow (host C++).
//
// The step-1 Jacobian J1 of every scenario shares one sparsity pattern, set
// by the Y_bus pattern and the bus-type partition (symbolic-analysis and
// BDE-layout passages of Sec. III-B).  This module builds, once per network:
//
//  * a fill-reducing elimination order of the non-slack buses (exact minimum
//    degree on the bus graph, ties to the lowest bus index);
//  * the 2x2-block pattern of L+U: every non-slack bus i owns the block
//    unknowns (theta_i, |V|_i) and the block equations (dP_i, dQ_i); on a PV
//    bus the |V| unknown and the dQ row are padding (identity diagonal, zero
//    coupling), so the block system has exactly the Newton solution;
//  * row-oriented ("up-looking") elimination lists: for each L block (a,k)
//    the row-relative targets in row a of the U blocks of row k;
//  * level sets for the factorisation / forward solve (dependencies on
//    earlier rows) and for the backward solve (dependencies on later rows);
//  * the position of the transposed block of every block (for the adjoint's
//    transposed solves), and the Y_bus entry that feeds every block (the
//    Jacobian fill map of the value-update kernel, Algorithm 1).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sable {

struct Symbolic {
  int32_t n_bus = 0;
  int32_t slack = -1;
  int32_t nb = 0;                    // block rows = non-slack buses
  std::vector<int32_t> bus_type;     // [n_bus] 0 PQ, 1 PV, 2 slack
  std::vector<int32_t> blk_bus;      // [nb] bus of block row a (elimination order)
  std::vector<int32_t> bus_blk;      // [n_bus] block row of a bus, -1 for the slack

  // Y_bus (CSR, columns sorted)
  std::vector<int32_t> y_rp, y_ci;
  std::vector<double> y_g, y_b;
  std::vector<int32_t> y_tr;         // [nnzY] position of the transposed entry

  // block L+U pattern, CSR over block rows in elimination order, sorted columns
  std::vector<int32_t> rp, ci, diag; // rp [nb+1], ci [nnzb], diag [nb]
  std::vector<int32_t> prow;         // [nnzb] block row of each position
  std::vector<int32_t> mirror;       // [nnzb] position of the transposed block
  std::vector<int32_t> lu_src;       // [nnzb] Y_bus entry of the block, -1 if fill-in

  // elimination lists: for L position p = (a,k): targets for U(k, >k)
  std::vector<int32_t> upd_start;    // [nnzb] (only L positions meaningful)
  std::vector<int32_t> upd_tgt;      // row-relative block offsets inside row a

  // level schedules
  std::vector<int32_t> lev_l_ptr, lev_l_rows;   // forward solve / U^T solve
  std::vector<int32_t> lev_u_ptr, lev_u_rows;   // backward solve / L^T solve

  // factorisation schedule, right-looking by levels with owner-computes rows:
  // at level h each row applies the elimination steps whose pivot row was
  // finished at level h-1 and, once its last pivot is in, inverts its own
  // pivot block.  Tasks of one level touch distinct rows.
  std::vector<int32_t> task_ptr;  // [n_levels_l + 1]
  std::vector<int32_t> task4;     // [n_tasks][4]: row a, first step, end step, finalise flag
  std::vector<int32_t> step4;     // [n_steps][4]: q = L position - rp[a], k, start of U(k,>k), |U(k,>k)|
  std::vector<int32_t> step_ts;   // [n_steps]: first entry of the step's targets in upd_tgt
  // dense tail: the last tail_t block rows (the top of the elimination tree,
  // highest levels) are factorised and solved by one wavefront per scenario
  // without workgroup barriers.  tail_pos[i*t + j] is the position of block
  // (tail_base + i, tail_base + j) or -1; tail_split[i] the first position of
  // tail row i whose column lies in the tail.  task_ptr covers the levels of
  // the barrier-synchronised part only; lev_um_* are the backward-solve
  // levels of the rows outside the tail.
  int32_t tail_t = 0, tail_base = 0, tail_h = 0;
  int32_t n_task_levels = 0, n_fs_levels = 0;
  std::vector<int32_t> tail_pos, tail_split;
  // structure of the tail block as bit masks over tail columns (tail_t <= 32):
  // tail_mask[k] bit j: block (k, j), j > k, of the tail is nonzero;
  // tail_mask[t] bit j: column j has a nonzero below the diagonal;
  // tail_mask[t + 1] bit j: column j has a nonzero above the diagonal
  std::vector<uint32_t> tail_mask;
  // compact numbering of the tail rows' blocks in tail columns (for a copy
  // of the tail in LDS): tail_cblk[c] is the position of compact block c;
  // compact index of position p of tail row l = tail_lbase[l] + (p - rp[tail_base + l]);
  // tail_cpos[i*t + j] = compact index of block (tail_base + i, tail_base + j) or -1
  std::vector<int32_t> tail_cblk, tail_lbase, tail_cpos;
  // elimination program of the tail pivots in the compact numbering, read
  // from LDS by the LDS copy of the tail.  Row/pivot k's record at 8k:
  // {compact index of its pivot block, compact index of its first block right
  // of the diagonal (the others follow), nu | ns << 16, offset of its step
  // words, offset of its update words, mask of its blocks left of the
  // diagonal (bit j: block (k, j) in the tail), mask of those right of it,
  // 0}.  Step words (ns): compact index of L(i, k) | (i - tail_base) << 16
  // for the rows i below with a block in column k.  Records and step words
  // form the prefix [0, tail_prog_prefix); the update words follow: ns * nu
  // per pivot, step by step, each target | L << 11 | j << 22 for target
  // (i, column of the j-th block right of the pivot), all compact indices
  // below 2048.  A row's blocks in tail columns have consecutive compact
  // indices in column order, so the masks locate each of them.
  std::vector<int32_t> tail_prog;
  int32_t tail_prog_prefix = 0;
  std::vector<int32_t> lev_um_ptr, lev_um_rows;
  // Jacobian fill record of every block: Y_bus entry (-1: fill-in), bus of
  // the row, bus of the column, flags (1 diagonal, 2 row bus PV, 4 column bus PV)
  std::vector<int32_t> fill4;     // [nnzb][4]

  // statistics
  int64_t nnz_j1 = 0;        // scalar nonzeros of J1 (real unknowns only)
  int64_t nnz_lu = 0;        // scalar nonzeros of L+U over real unknowns
  int64_t n_upd = 0;         // block multiply-subtract operations per factorisation
  double factor_flops = 0;   // scalar flops of one factorisation on 2x2 blocks
  int32_t max_row_blocks = 0;
  int32_t n_pv = 0, n_pq = 0;

  int32_t nnzb() const { return (int32_t)ci.size(); }
  int32_t n_levels_l() const { return (int32_t)lev_l_ptr.size() - 1; }
  int32_t n_levels_u() const { return (int32_t)lev_u_ptr.size() - 1; }
};

// Level schedules cut into chunks whose metadata a workgroup copies into LDS
// before working through it (HBM-resident slices, where every dependent
// metadata load would otherwise be an L2 round trip).  A chunk holds whole
// tasks (rows) of one level; chunks follow level order; each chunk is a run
// of int32 padded to a multiple of 4:
//  factor:  [ntask, nstep, ntgt, 0], ntask + 1 task records {row, rp[row],
//           diag[row] - rp[row] if the row inverts its pivot block else -1,
//           first step}, nstep + 1 step records {L position - rp[row], pivot
//           row, first position of the pivot's U row right of the diagonal,
//           first target}, ntgt row-relative target positions;
//  solves:  [nrow, ncol, 0, 0], nrow + 1 row records {row, first position,
//           0, first column}, ncol column indices (forward: the L part of
//           each row, backward: the U part right of the diagonal).
// The trailing record of each list only carries the end index.
//  transposed solves (adjoint): as the solves, with a pair (column,
//           position of the transposed block) per entry: U^T by the forward
//           levels over the L part of each row, L^T by the backward levels
//           over the U part.
struct LevelChunks {
  std::vector<int32_t> f_ptr, f_blob;     // factor tasks
  std::vector<int32_t> fs_ptr, fs_blob;   // forward solve, rows outside the tail
  std::vector<int32_t> bs_ptr, bs_blob;   // backward solve, rows outside the tail
  std::vector<int32_t> ut_ptr, ut_blob;   // U^T solve, rows outside the tail
  std::vector<int32_t> lt_ptr, lt_blob;   // L^T solve, rows outside the tail
  // U^T terms of the tail rows on rows outside the tail: for tail row l the
  // pairs (column k, position of block (k, tail_base + l)), [tt_ptr[l], tt_ptr[l+1])
  std::vector<int32_t> tt_ptr, tt_pairs;
  int32_t max_ints = 0;                   // largest chunk, int32 words
};

// budget_ints: largest chunk in int32 words.  Returns 0, or PF_EINVAL if a
// single row does not fit the budget.
int build_level_chunks(const Symbolic& S, int32_t budget_ints, LevelChunks& out, std::string& err);

// Returns 0 on success; on failure a negative PF_E* code and a message.
// tail_max: largest dense tail (0 disables it; at most 64)
int analyze(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
            const int32_t* y_indices, const double* y_g, const double* y_b,
            Symbolic& out, std::string& err, int32_t tail_max = 32);

// pi-model branch admittances assembled into CSR (columns sorted, duplicate
// branches summed).  Returns nnz, or a negative error code.
int ybus_from_branches(int32_t n_bus, int32_t n_branch, const int32_t* f, const int32_t* t,
                       const double* r, const double* x, const double* bc,
                       std::vector<int32_t>& rp, std::vector<int32_t>& ci,
                       std::vector<double>& g, std::vector<double>& b, std::string& err);

}  // namespace sable
