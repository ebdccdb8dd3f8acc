// Host-side validation of the factorisation and triangular-solve schedules
// that the symbolic pass builds (one-time symbolic analysis, Sec. III-B).
// Test support only: built by tests/test_host_schedule.py with
// -fsanitize=address,undefined together with the library's host modules
// (symbolic.cpp, operators.cpp), so the sanitizers cover them on every grid.
//
// The device kernels run every level of a schedule as one barrier-separated
// pass ("epoch" below: one metadata chunk), and inside a pass a group of
// lanes of one wavefront owns one row.  This program replays that order on
// the host and checks:
//  * structure: the block pattern is closed under elimination, every L block
//    of a row outside the dense tail is eliminated by exactly one step,
//    every such row inverts its pivot block exactly once, and the step and
//    target records point where the pattern says;
//  * levels: each chunk holds rows of one level only, levels never decrease
//    from chunk to chunk, and the rows of one chunk are distinct;
//  * ordering across passes: every value a task reads outside its own row
//    (the pivot row's U blocks, its inverted pivot block and its forward
//    right-hand side) and every multiplier it forms was last written in an
//    earlier pass, and nothing writes it again later;
//  * ordering inside a task: with E lanes per scenario on a task (E = 1 .. 64
//    for every launch shape), a value written by one lane and later read or
//    written by another lane of the same wavefront is separated by a fence
//    (the kernel's rule: a fence between successive steps whenever E > 1,
//    and before the pivot inversion only after a task of several steps).
//    A single-step task needs none: the pivot of each step of a task that
//    inverts its row's pivot block is a child of the row in the elimination
//    tree, so the row's diagonal is the first target of that step, updated
//    by lane 0, the lane that inverts it; the program checks that property;
//  * the forward and backward solve schedules read only unknowns solved in
//    earlier passes (or by the dense tail, which the backward solve runs
//    first), and the transposed schedules of the adjoint mirror them;
//  * the dense tail's per-pivot step lists cover its internal L blocks in
//    pivot order, and its structure masks match its pattern;
//  * every Jacobian fill record names the Y_bus entry of its bus pair.
//
// Option --variant-fill-inverts-level0 replays a variant in which the pivot
// blocks of the rows without L blocks are inverted by the Jacobian fill,
// before its closing barrier, and the factor schedule starts one level
// later.
//
// Input (text): n_bus n_branch, then n_bus bus types, then n_branch lines
// "from to r x b".  Output: one summary line; exit status 0 when every check
// holds, 1 with the first violations printed otherwise.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "operators.h"
#include "sable_pf.h"
#include "symbolic.h"

using sable::LevelChunks;
using sable::Symbolic;

namespace {

int g_fail = 0;

#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      if (g_fail < 20) {                                  \
        std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
        std::fprintf(stderr, __VA_ARGS__);                \
        std::fprintf(stderr, "\n");                       \
      }                                                   \
      ++g_fail;                                           \
    }                                                     \
  } while (0)

struct Factor {   // one decoded factor chunk
  struct Task { int row, rp, diagoff, s0, s1; };
  struct Step { int q, k, ustart, t0, t1; };
  std::vector<Task> tasks;
  std::vector<Step> steps;
  std::vector<int> tgt;
};

std::vector<Factor> decode_factor(const LevelChunks& C) {
  std::vector<Factor> out;
  for (size_t c = 0; c + 1 < C.f_ptr.size(); ++c) {
    const int* h = C.f_blob.data() + C.f_ptr[c];
    const int nt = h[0], ns = h[1], ng = h[2];
    const int* tk = h + 4;
    const int* st = tk + 4 * (nt + 1);
    const int* tg = st + 4 * (ns + 1);
    Factor F;
    for (int i = 0; i < nt; ++i)
      F.tasks.push_back({tk[4 * i], tk[4 * i + 1], tk[4 * i + 2], tk[4 * i + 3], tk[4 * (i + 1) + 3]});
    for (int i = 0; i < ns; ++i)
      F.steps.push_back({st[4 * i], st[4 * i + 1], st[4 * i + 2], st[4 * i + 3], st[4 * (i + 1) + 3]});
    F.tgt.assign(tg, tg + ng);
    CHECK(st[4 * ns + 3] == ng, "factor chunk %zu: target count %d != %d", c, st[4 * ns + 3], ng);
    CHECK(tk[4 * nt + 3] == ns, "factor chunk %zu: step count", c);
    CHECK(C.f_ptr[c] + 4 + 4 * (nt + 1) + 4 * (ns + 1) + ng <= C.f_ptr[c + 1], "factor chunk %zu overflows", c);
    CHECK(C.f_ptr[c + 1] - C.f_ptr[c] <= C.max_ints, "factor chunk %zu above max_ints", c);
    out.push_back(F);
  }
  return out;
}

struct Solve {   // one decoded solve chunk (pairs: transposed schedules)
  struct Row { int row, p0; std::vector<int> col, pos; };
  std::vector<Row> rows;
};

std::vector<Solve> decode_solve(const std::vector<int32_t>& ptr, const std::vector<int32_t>& blob, bool pairs,
                                int max_ints) {
  std::vector<Solve> out;
  const int w = pairs ? 2 : 1;
  for (size_t c = 0; c + 1 < ptr.size(); ++c) {
    const int* h = blob.data() + ptr[c];
    const int nr = h[0], nc = h[1];
    const int* rw = h + 4;
    const int* cols = rw + 4 * (nr + 1);
    Solve S;
    for (int i = 0; i < nr; ++i) {
      Solve::Row r{rw[4 * i], rw[4 * i + 1], {}, {}};
      for (int j = rw[4 * i + 3]; j < rw[4 * (i + 1) + 3]; ++j) {
        r.col.push_back(cols[w * j]);
        if (pairs) r.pos.push_back(cols[w * j + 1]);
      }
      S.rows.push_back(r);
    }
    CHECK(rw[4 * nr + 3] == nc, "solve chunk %zu: column count", c);
    CHECK(ptr[c] + 4 + 4 * (nr + 1) + w * nc <= ptr[c + 1], "solve chunk %zu overflows", c);
    CHECK(ptr[c + 1] - ptr[c] <= max_ints, "solve chunk %zu above max_ints", c);
    out.push_back(S);
  }
  return out;
}

// the level of a factor chunk: steps eliminate pivots of level h - 1, the
// rows that invert their pivot block sit at level h
int factor_chunk_level(const Symbolic& S, const std::vector<int>& lev, const Factor& F, size_t c) {
  int h = -1;
  for (const auto& t : F.tasks) {
    for (int i = t.s0; i < t.s1; ++i) {
      const int hk = lev[F.steps[i].k] + 1;
      CHECK(h < 0 || h == hk, "factor chunk %zu mixes levels %d and %d", c, h, hk);
      h = hk;
    }
    if (t.diagoff >= 0) {
      CHECK(h < 0 || h == lev[t.row], "factor chunk %zu: a row of level %d inverts at level %d", c, lev[t.row], h);
      h = lev[t.row];
    }
  }
  (void)S;
  return h;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s network.txt [--budget N] [--tail N] [--variant-fill-inverts-level0]\n",
                 argv[0]);
    return 2;
  }
  int budget = 12288, tail_max = 32;
  bool variant = false;
  for (int i = 2; i < argc; ++i) {
    if (!std::strcmp(argv[i], "--budget") && i + 1 < argc) budget = std::atoi(argv[++i]);
    else if (!std::strcmp(argv[i], "--tail") && i + 1 < argc) tail_max = std::atoi(argv[++i]);
    else if (!std::strcmp(argv[i], "--variant-fill-inverts-level0")) variant = true;
    else { std::fprintf(stderr, "unknown option %s\n", argv[i]); return 2; }
  }
  FILE* fp = std::fopen(argv[1], "r");
  if (!fp) { std::perror(argv[1]); return 2; }
  int n = 0, m = 0;
  if (std::fscanf(fp, "%d %d", &n, &m) != 2 || n < 2 || m < 0) { std::fprintf(stderr, "bad header\n"); return 2; }
  std::vector<int32_t> bt(n), f(m), t(m);
  std::vector<double> r(m), x(m), bc(m);
  for (int i = 0; i < n; ++i)
    if (std::fscanf(fp, "%d", &bt[i]) != 1) { std::fprintf(stderr, "bad bus types\n"); return 2; }
  for (int k = 0; k < m; ++k)
    if (std::fscanf(fp, "%d %d %lf %lf %lf", &f[k], &t[k], &r[k], &x[k], &bc[k]) != 5) {
      std::fprintf(stderr, "bad branch %d\n", k);
      return 2;
    }
  std::fclose(fp);

  std::vector<int32_t> yrp, yci;
  std::vector<double> yg, yb;
  std::string err;
  if (sable::ybus_from_branches(n, m, f.data(), t.data(), r.data(), x.data(), bc.data(), yrp, yci, yg, yb, err) < 0) {
    std::fprintf(stderr, "ybus: %s\n", err.c_str());
    return 2;
  }
  Symbolic S;
  if (sable::analyze(n, bt.data(), yrp.data(), yci.data(), yg.data(), yb.data(), S, err, tail_max) != 0) {
    std::fprintf(stderr, "analyze: %s\n", err.c_str());
    return 2;
  }
  LevelChunks C;
  if (sable::build_level_chunks(S, budget, C, err) != 0) {
    std::fprintf(stderr, "chunks: %s\n", err.c_str());
    return 2;
  }
  sable::OperatorSet ops;
  if (sable::build_operators(n, bt.data(), S.y_rp.data(), S.y_ci.data(), ops, err) != 0) {
    std::fprintf(stderr, "operators: %s\n", err.c_str());
    return 2;
  }

  const int nb = S.nb, tb = S.tail_base, nnzb = S.nnzb();
  auto pos_of = [&](int a, int j) -> int {   // position of block (a, j) or -1
    for (int p = S.rp[a]; p < S.rp[a + 1]; ++p)
      if (S.ci[p] == j) return p;
    return -1;
  };

  // ---- pattern: sorted rows, diagonal, closed under elimination
  for (int a = 0; a < nb; ++a) {
    CHECK(S.ci[S.diag[a]] == a, "row %d: diagonal", a);
    for (int p = S.rp[a]; p + 1 < S.rp[a + 1]; ++p) CHECK(S.ci[p] < S.ci[p + 1], "row %d unsorted", a);
    for (int p = S.rp[a]; p < S.diag[a]; ++p) {
      const int k = S.ci[p];
      for (int q = S.diag[k] + 1; q < S.rp[k + 1]; ++q)
        CHECK(pos_of(a, S.ci[q]) >= 0, "fill of (%d, %d) through pivot %d missing", a, S.ci[q], k);
    }
  }
  std::vector<int> lev(nb, 0);
  for (int a = 0; a < nb; ++a)
    for (int p = S.rp[a]; p < S.diag[a]; ++p) lev[a] = std::max(lev[a], lev[S.ci[p]] + 1);

  // ---- factor schedule
  std::vector<Factor> FC = decode_factor(C);
  if (variant) {
    // the fill inverts the pivot blocks of the rows without L blocks (level
    // 0), so those tasks leave the schedule
    for (auto& F : FC) {
      std::vector<Factor::Task> keep;
      for (const auto& tk : F.tasks)
        if (!(tk.s0 == tk.s1 && tk.diagoff >= 0 && lev[tk.row] == 0)) keep.push_back(tk);
      F.tasks.swap(keep);
    }
  }
  std::vector<int> step_of(nnzb, 0), fin_of(nb, 0);
  // epoch of the last write of every block position, of every dinv / y row;
  // the fill is epoch 0, factor chunk c is epoch c + 1
  std::vector<int> w_pos(nnzb, 0), w_dinv(nb, -1), w_y(nb, 0);
  std::vector<int> pos_read_last(nnzb, -1);   // last epoch a multiplier (L block) was read
  // reads of a pivot row (its U blocks, inverted pivot and right-hand side)
  // by epoch, and the last epoch anything writes into a row
  std::vector<std::pair<int, int>> row_reads;
  std::vector<int> row_last_write(nb, 0);
  if (variant)
    for (int a = 0; a < nb; ++a)
      if (lev[a] == 0 && a < tb) { w_dinv[a] = 0; fin_of[a]++; }
  int prev_level = -1;
  long hazards_intra = 0, tasks = 0;
  for (size_t c = 0; c < FC.size(); ++c) {
    const Factor& F = FC[c];
    const int e = (int)c + 1;
    const int h = factor_chunk_level(S, lev, F, c);
    CHECK(h >= prev_level, "factor chunk %zu: level %d after level %d", c, h, prev_level);
    prev_level = h;
    std::set<int> rows_here;
    for (const auto& tk : F.tasks) {
      CHECK(rows_here.insert(tk.row).second, "factor chunk %zu: row %d twice", c, tk.row);
      CHECK(tk.row >= 0 && tk.row < nb && tk.rp == S.rp[tk.row], "factor chunk %zu: bad task record", c);
    }
    for (const auto& tk : F.tasks) {
      const int a = tk.row;
      ++tasks;
      // structure and cross-pass ordering
      for (int i = tk.s0; i < tk.s1; ++i) {
        const Factor::Step& s = F.steps[i];
        const int p = S.rp[a] + s.q, k = s.k;
        CHECK(p >= S.rp[a] && p < S.diag[a] && S.ci[p] == k, "task row %d: step %d is not L(%d,%d)", a, i, a, k);
        CHECK(k < tb, "task row %d: pivot %d inside the tail", a, k);
        CHECK(s.ustart == S.diag[k] + 1 && s.t1 - s.t0 == S.rp[k + 1] - s.ustart,
              "task row %d pivot %d: U row record", a, k);
        step_of[p]++;
        CHECK(!rows_here.count(k), "pivot row %d is a task of the same pass as row %d", k, a);
        CHECK(w_dinv[k] >= 0 && w_dinv[k] < e, "row %d reads dinv[%d] before it is written", a, k);
        CHECK(w_y[k] < e, "row %d reads y[%d] written in the same pass", a, k);
        for (int q = s.ustart; q < S.rp[k + 1]; ++q) CHECK(w_pos[q] < e, "row %d reads U(%d,.) of this pass", a, k);
        CHECK(w_pos[p] < e, "multiplier (%d,%d) updated in its own pass", a, k);
        pos_read_last[p] = e;
        row_reads.push_back({k, e});
        std::set<int> distinct;
        for (int j = s.t0; j < s.t1; ++j) {
          const int off = F.tgt[j];
          const int tp = S.rp[a] + off;
          CHECK(off >= 0 && tp < S.rp[a + 1], "row %d: target offset out of the row", a);
          CHECK(S.ci[tp] == S.ci[s.ustart + (j - s.t0)], "row %d: target column mismatch", a);
          CHECK(distinct.insert(tp).second, "row %d: a step with a repeated target", a);
          CHECK(pos_read_last[tp] < 0 || tp >= S.diag[a],
                "row %d: target (%d,%d) updated after its multiplier was formed", a, a, S.ci[tp]);
          w_pos[tp] = e;
        }
        w_pos[p] = e;   // the multiplier itself
        w_y[a] = e;
        row_last_write[a] = e;
      }
      if (tk.diagoff >= 0) {
        CHECK(tk.diagoff == S.diag[a] - S.rp[a], "row %d: pivot record", a);
        for (int i = tk.s0; i < tk.s1; ++i)   // each pivot is a child of row a: the diagonal comes first
          CHECK(F.steps[i].t1 > F.steps[i].t0 && F.tgt[F.steps[i].t0] == tk.diagoff,
                "row %d: pivot %d is not its child in the elimination tree", a, F.steps[i].k);
        CHECK(a < tb, "tail row %d inverts in the level schedule", a);
        fin_of[a]++;
        w_dinv[a] = e;
        row_last_write[a] = e;
      }
      // ordering inside the task: phases = steps, then the pivot inversion;
      // lane of target j of a step: j mod E; multipliers and the inversion:
      // lane 0.  A value written by lane x and touched later by lane y != x
      // needs a fence in between.
      const int nsteps = tk.s1 - tk.s0;
      for (int E = 1; E <= 64; E *= 2) {
        std::vector<int> owner(S.rp[a + 1] - S.rp[a], -1), wphase(S.rp[a + 1] - S.rp[a], -1);
        auto fenced = [&](int from, int to) {   // a fence between phase `from` and phase `to` > from
          if (E == 1) return false;
          if (to < nsteps) return true;              // between successive steps
          return nsteps > 1;                         // before the pivot inversion
        };
        bool bad = false;
        auto touch = [&](int off, int lane, int ph, bool write) {
          if (owner[off] >= 0 && owner[off] != lane && wphase[off] < ph && !fenced(wphase[off], ph)) bad = true;
          if (write) { owner[off] = lane; wphase[off] = ph; }
        };
        for (int i = tk.s0; i < tk.s1; ++i) {
          const Factor::Step& s = F.steps[i];
          const int ph = i - tk.s0;
          for (int l = 0; l < E; ++l) touch(s.q, l, ph, false);   // every lane reads the multiplier
          for (int j = s.t0; j < s.t1; ++j) touch(F.tgt[j], (j - s.t0) % E, ph, true);
          touch(s.q, 0, ph, true);
        }
        if (tk.diagoff >= 0) touch(tk.diagoff, 0, nsteps, false);
        if (bad) { ++hazards_intra; break; }
      }
    }
  }
  CHECK(hazards_intra == 0, "%ld tasks with unfenced lane-to-lane reuse", hazards_intra);
  for (const auto& rr : row_reads)
    CHECK(row_last_write[rr.first] < rr.second, "pivot row %d read in pass %d, written again in pass %d",
          rr.first, rr.second, row_last_write[rr.first]);
  for (int a = 0; a < nb; ++a) {
    for (int p = S.rp[a]; p < S.diag[a]; ++p) {
      const bool levelled = S.ci[p] < tb;
      CHECK(step_of[p] == (levelled ? 1 : 0), "L(%d,%d) eliminated %d times", a, S.ci[p], step_of[p]);
    }
    CHECK(fin_of[a] == (a < tb ? 1 : 0), "row %d inverts its pivot %d times", a, fin_of[a]);
  }
  // after the levelled part every tail row's blocks outside tail columns are final
  const int e_end = (int)FC.size() + 1;
  for (int a = tb; a < nb; ++a)
    for (int p = S.rp[a]; p < S.tail_split[a - tb]; ++p) CHECK(w_pos[p] < e_end, "tail row %d", a);

  // ---- dense tail: the elimination program of the LDS tail copy and masks
  const int tt = S.tail_t;
  {
    const int nblk = (int)S.tail_cblk.size();
    auto cidx = [&](int a, int p) { return S.tail_lbase[a - tb] + (p - S.rp[a]); };
    auto rec = [&](int k, int f) { return S.tail_prog[8 * k + f]; };
    std::vector<int> cover(nnzb, 0);
    CHECK(S.tail_prog.size() >= 8 * (size_t)tt && S.tail_prog_prefix >= 8 * tt &&
          (size_t)S.tail_prog_prefix <= S.tail_prog.size(), "tail program extent");
    for (int k = 0; k < tt && !S.tail_prog.empty(); ++k) {
      const int ak = tb + k;
      const int dk = rec(k, 0), ks = rec(k, 1), nu = rec(k, 2) & 0xffff, ns = rec(k, 2) >> 16;
      const int soff = rec(k, 3), uoff = rec(k, 4);
      const unsigned lm = (unsigned)rec(k, 5), um = (unsigned)rec(k, 6);
      CHECK(dk == cidx(ak, S.diag[ak]) && S.tail_cblk[dk] == S.diag[ak], "tail program pivot %d", k);
      CHECK(nu == S.rp[ak + 1] - S.diag[ak] - 1, "tail program pivot %d: U count", k);
      CHECK(nu == 0 || ks == dk + 1, "tail program pivot %d: first U", k);
      CHECK(soff + ns <= S.tail_prog_prefix, "tail program pivot %d: steps outside the prefix", k);
      CHECK(uoff >= S.tail_prog_prefix && uoff + (size_t)ns * nu <= S.tail_prog.size(),
            "tail program pivot %d: updates extent", k);
      // masks: the row's blocks in tail columns have consecutive compact
      // indices in column order, L part, pivot, U part
      int rank = 0;
      for (int j = 0; j < tt; ++j) {
        const int cp = S.tail_cpos[(size_t)k * tt + j];
        const bool inl = (lm >> j) & 1u, inu = (um >> j) & 1u;
        CHECK(inl == (cp >= 0 && j < k) && inu == (cp >= 0 && j > k), "tail masks row %d col %d", k, j);
        if (cp >= 0) {
          CHECK(cp == dk - __builtin_popcount(lm) + rank, "tail row %d: compact order at col %d", k, j);
          ++rank;
        }
      }
      CHECK(__builtin_popcount(um) == nu, "tail row %d: U mask count", k);
      std::set<int> targets, lus;
      for (int j = 0; j < nu; ++j) lus.insert(ks + j);
      lus.insert(dk);
      for (int si = 0; si < ns; ++si) {
        const int w = S.tail_prog[soff + si], lc = w & 0xffff, ir = w >> 16;
        const int a = tb + ir;
        CHECK(ir > k && ir < tt, "tail program pivot %d: step row %d", k, ir);
        if (!(ir > k && ir < tt)) continue;
        const int p = S.tail_cblk[lc];
        CHECK(lc >= 0 && lc < nblk && S.prow[p] == a && S.ci[p] == ak && p < S.diag[a],
              "tail program pivot %d: L block of row %d", k, ir);
        cover[p]++;
        lus.insert(lc);
        for (int j = 0; j < nu; ++j) {
          const unsigned r = (unsigned)S.tail_prog[uoff + (size_t)si * nu + j];
          const int tg = (int)(r & 2047u), l2 = (int)((r >> 11) & 2047u), jj = (int)(r >> 22);
          const int col = S.ci[S.diag[ak] + 1 + j];
          int want = -1;
          for (int q = S.rp[a]; q < S.rp[a + 1]; ++q)
            if (S.ci[q] == col) want = cidx(a, q);
          CHECK(l2 == lc && jj == j && tg == want && want >= 0, "tail program pivot %d: update (%d, %d)", k, ir, j);
          CHECK(targets.insert(tg).second, "tail program pivot %d: target twice", k);
        }
      }
      for (int tg : targets) CHECK(!lus.count(tg), "tail program pivot %d: target is an operand", k);
    }
    for (int a = tb; a < nb; ++a)
      for (int p = S.rp[a]; p < S.diag[a]; ++p)
        if (S.ci[p] >= tb) CHECK(cover[p] == 1, "tail L(%d,%d) covered %d times", a, S.ci[p], cover[p]);
    // numeric replay: the program's factorisation and the mask-walking
    // triangular solves on random values of the tail pattern, against a
    // dense right-looking block LU and dense solves of the same t x t block
    // matrix
    if (tt > 0 && !S.tail_prog.empty()) {
      using B4 = std::array<double, 4>;
      std::mt19937_64 rng(7);
      std::uniform_real_distribution<double> U(-1.0, 1.0);
      std::vector<B4> v(nblk), A((size_t)tt * tt, {0, 0, 0, 0}), dinv(tt);
      for (int i = 0; i < tt; ++i)
        for (int j = 0; j < tt; ++j) {
          const int cp = S.tail_cpos[(size_t)i * tt + j];
          if (cp < 0) continue;
          B4 b = {U(rng), U(rng), U(rng), U(rng)};
          if (i == j) { b[0] += 4.0 * tt; b[3] += 4.0 * tt; }
          v[cp] = b;
          A[(size_t)i * tt + j] = b;
        }
      auto mul = [](const B4& x, const B4& y) {
        return B4{x[0] * y[0] + x[1] * y[2], x[0] * y[1] + x[1] * y[3], x[2] * y[0] + x[3] * y[2],
                  x[2] * y[1] + x[3] * y[3]};
      };
      auto inv = [](const B4& x) {
        const double d = x[0] * x[3] - x[1] * x[2];
        return B4{x[3] / d, -x[1] / d, -x[2] / d, x[0] / d};
      };
      for (int k = 0; k < tt; ++k) {
        const int dk = rec(k, 0), ks = rec(k, 1), nu = rec(k, 2) & 0xffff, ns = rec(k, 2) >> 16;
        const B4 Di = inv(v[dk]);
        dinv[k] = Di;
        for (size_t q = 0; q < (size_t)ns * nu; ++q) {
          const unsigned r = (unsigned)S.tail_prog[rec(k, 4) + q];
          const B4 M = mul(mul(v[(r >> 11) & 2047u], Di), v[ks + (r >> 22)]);
          for (int e = 0; e < 4; ++e) v[r & 2047u][e] -= M[e];
        }
        for (int si = 0; si < ns; ++si) {
          const int lc = S.tail_prog[rec(k, 3) + si] & 0xffff;
          v[lc] = mul(v[lc], Di);
        }
        const B4 Dd = inv(A[(size_t)k * tt + k]);
        for (int i = k + 1; i < tt; ++i) {
          const B4 L = mul(A[(size_t)i * tt + k], Dd);
          for (int j = k + 1; j < tt; ++j) {
            const B4 M = mul(L, A[(size_t)k * tt + j]);
            for (int e = 0; e < 4; ++e) A[(size_t)i * tt + j][e] -= M[e];
          }
          A[(size_t)i * tt + k] = L;
        }
      }
      double worst = 0.0;
      for (int i = 0; i < tt; ++i)
        for (int j = 0; j < tt; ++j) {
          const int cp = S.tail_cpos[(size_t)i * tt + j];
          for (int e = 0; e < 4; ++e) {
            const double ref = A[(size_t)i * tt + j][e];
            const double got = cp < 0 ? 0.0 : v[cp][e];
            worst = std::max(worst, std::fabs(got - ref) / (1.0 + std::fabs(ref)));
          }
        }
      CHECK(worst < 1e-12, "tail program replay differs from a dense LU by %g", worst);
      // solves: row i walks its blocks by its masks (forward: lowest column
      // first, backward: highest first), as the lanes do
      std::vector<double> y(2 * tt), ref(2 * tt);
      for (auto& x : y) x = U(rng);
      ref = y;
      for (int k = 0; k < tt; ++k)
        for (int i = k + 1; i < tt; ++i) {
          const B4& L = A[(size_t)i * tt + k];
          ref[2 * i] -= L[0] * ref[2 * k] + L[1] * ref[2 * k + 1];
          ref[2 * i + 1] -= L[2] * ref[2 * k] + L[3] * ref[2 * k + 1];
        }
      for (int j = tt - 1; j >= 0; --j) {
        const B4 D = inv(A[(size_t)j * tt + j]);
        const double x0 = D[0] * ref[2 * j] + D[1] * ref[2 * j + 1], x1 = D[2] * ref[2 * j] + D[3] * ref[2 * j + 1];
        ref[2 * j] = x0;
        ref[2 * j + 1] = x1;
        for (int i = 0; i < j; ++i) {
          const B4& Ub = A[(size_t)i * tt + j];
          ref[2 * i] -= Ub[0] * x0 + Ub[1] * x1;
          ref[2 * i + 1] -= Ub[2] * x0 + Ub[3] * x1;
        }
      }
      for (int k = 0; k < tt; ++k) {   // forward, in pivot order
        for (int i = k + 1; i < tt; ++i) {
          const unsigned lm = (unsigned)rec(i, 5);
          if (!((lm >> k) & 1u)) continue;
          const int idx = rec(i, 0) - __builtin_popcount(lm) + __builtin_popcount(lm & ((1u << k) - 1u));
          const B4& L = v[idx];
          y[2 * i] -= L[0] * y[2 * k] + L[1] * y[2 * k + 1];
          y[2 * i + 1] -= L[2] * y[2 * k] + L[3] * y[2 * k + 1];
        }
      }
      for (int j = tt - 1; j >= 0; --j) {
        const B4& D = dinv[j];
        const double x0 = D[0] * y[2 * j] + D[1] * y[2 * j + 1], x1 = D[2] * y[2 * j] + D[3] * y[2 * j + 1];
        y[2 * j] = x0;
        y[2 * j + 1] = x1;
        for (int i = 0; i < j; ++i) {
          const unsigned um = (unsigned)rec(i, 6);
          if (!((um >> j) & 1u)) continue;
          const int idx = rec(i, 0) + __builtin_popcount(um & ((j < 31 ? (2u << j) : 0u) - 1u));
          const B4& Ub = v[idx];
          y[2 * i] -= Ub[0] * x0 + Ub[1] * x1;
          y[2 * i + 1] -= Ub[2] * x0 + Ub[3] * x1;
        }
      }
      double werr = 0.0;
      for (int i = 0; i < 2 * tt; ++i) werr = std::max(werr, std::fabs(y[i] - ref[i]) / (1.0 + std::fabs(ref[i])));
      CHECK(werr < 1e-12, "tail solves differ from dense solves by %g", werr);
      printf("tail_replay_err %.3g solve_err %.3g over %d pivots, %d blocks, program %zu words (prefix %d)\n",
             worst, werr, tt, nblk, S.tail_prog.size(), S.tail_prog_prefix);
    }
    if (tt > 0 && tt <= 32)
      for (int i = 0; i < tt; ++i)
        for (int j = 0; j < tt; ++j) {
          const bool nz = S.tail_pos[(size_t)i * tt + j] >= 0 && i != j;
          if (j > i) CHECK(((S.tail_mask[i] >> j) & 1u) == (nz ? 1u : 0u), "tail mask row %d col %d", i, j);
          if (nz && j < i) CHECK((S.tail_mask[tt] >> j) & 1u, "tail lower mask col %d", j);
          if (nz && j > i) CHECK((S.tail_mask[tt + 1] >> j) & 1u, "tail upper mask col %d", j);
        }
  }

  // ---- solve schedules outside the tail
  auto solves = [&](const std::vector<int32_t>& ptr, const std::vector<int32_t>& blob, bool lower,
                    bool pairs, const char* name, std::vector<Solve>& out) {
    out = decode_solve(ptr, blob, pairs, C.max_ints);
    std::vector<int> done(nb, -1), seen(nb, 0);
    if (!lower)
      for (int a = tb; a < nb; ++a) done[a] = 0;   // the tail is solved first
    for (size_t c = 0; c < out.size(); ++c) {
      const int e = (int)c + 1;
      std::set<int> here;
      for (const auto& r : out[c].rows) CHECK(here.insert(r.row).second, "%s chunk %zu: row twice", name, c);
      for (const auto& r : out[c].rows) {
        const int a = r.row;
        CHECK(a >= 0 && a < tb, "%s: row %d outside the levelled part", name, a);
        seen[a]++;
        const int p0 = lower ? S.rp[a] : S.diag[a] + 1, p1 = lower ? S.diag[a] : S.rp[a + 1];
        CHECK(r.p0 == p0 && (int)r.col.size() == p1 - p0, "%s: row %d record", name, a);
        for (size_t j = 0; j < r.col.size(); ++j) {
          const int k = r.col[j];
          CHECK(k == S.ci[p0 + (int)j], "%s: row %d column %zu", name, a, j);
          CHECK(done[k] >= 0 && done[k] < e, "%s: row %d reads unknown %d before it is solved", name, a, k);
          if (pairs) {
            const int mp = r.pos[j];
            CHECK(mp >= 0 && mp < nnzb && S.prow[mp] == k && S.ci[mp] == a, "%s: mirror of (%d,%d)", name, a, k);
            CHECK(S.mirror[mp] == p0 + (int)j, "%s: mirror is not an involution at (%d,%d)", name, a, k);
          }
        }
      }
      for (const auto& r : out[c].rows) done[r.row] = e;
    }
    for (int a = 0; a < tb; ++a) CHECK(seen[a] == 1, "%s: row %d solved %d times", name, a, seen[a]);
  };
  std::vector<Solve> fs, bs, ut, lt;
  solves(C.fs_ptr, C.fs_blob, true, false, "forward", fs);
  solves(C.bs_ptr, C.bs_blob, false, false, "backward", bs);
  solves(C.ut_ptr, C.ut_blob, true, true, "U^T", ut);
  solves(C.lt_ptr, C.lt_blob, false, true, "L^T", lt);
  // the transposed schedules walk the same rows in the same order (their
  // passes may be cut differently: their records are twice as long)
  auto same_rows = [&](const std::vector<Solve>& A, const std::vector<Solve>& B, const char* name) {
    std::vector<const Solve::Row*> ra, rb;
    for (const auto& c : A) for (const auto& r : c.rows) ra.push_back(&r);
    for (const auto& c : B) for (const auto& r : c.rows) rb.push_back(&r);
    CHECK(ra.size() == rb.size(), "%s: %zu rows against %zu", name, ra.size(), rb.size());
    for (size_t i = 0; i < std::min(ra.size(), rb.size()); ++i)
      CHECK(ra[i]->row == rb[i]->row && ra[i]->col == rb[i]->col, "%s: row %zu differs", name, i);
  };
  same_rows(fs, ut, "U^T vs forward");
  same_rows(bs, lt, "L^T vs backward");
  // forward levels: every level strictly after the levels of the rows it reads
  for (int l = 0; l < tt; ++l) {
    const int a = tb + l;
    int q = C.tt_ptr[l];
    for (int p = S.rp[a]; p < S.tail_split[l]; ++p, ++q) {
      CHECK(S.ci[p] < tb && C.tt_pairs[2 * q] == S.ci[p] && C.tt_pairs[2 * q + 1] == S.mirror[p],
            "tail row %d: transposed term", a);
    }
    CHECK(q == C.tt_ptr[l + 1], "tail row %d: transposed term count", a);
  }

  // ---- Jacobian fill records
  std::vector<int> ycover(S.y_ci.size(), 0);
  for (int p = 0; p < nnzb; ++p) {
    const int a = S.prow[p], j = S.ci[p];
    const int bi = S.blk_bus[a], bj = S.blk_bus[j];
    const int yq = S.fill4[4 * p];
    CHECK(S.fill4[4 * p + 1] == bi && S.fill4[4 * p + 2] == bj, "fill record %d: buses", p);
    const int fl = (a == j ? 1 : 0) | (bt[bi] == PF_BUS_PV ? 2 : 0) | (bt[bj] == PF_BUS_PV ? 4 : 0);
    CHECK(S.fill4[4 * p + 3] == fl, "fill record %d: flags", p);
    if (yq >= 0) {
      CHECK(S.y_ci[yq] == bj && yq >= S.y_rp[bi] && yq < S.y_rp[bi + 1], "fill record %d: Y entry", p);
      ycover[yq]++;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int q = S.y_rp[i]; q < S.y_rp[i + 1]; ++q) {
      const bool inner = i != S.slack && S.y_ci[q] != S.slack;
      CHECK(ycover[q] == (inner ? 1 : 0), "Y entry (%d,%d) feeds %d blocks", i, S.y_ci[q], ycover[q]);
    }

  std::printf("buses %d blocks %d nnzb %d levels %d tail %d factor_passes %zu forward_passes %zu "
              "backward_passes %zu tasks %ld intra_task_hazards %ld violations %d\n",
              n, nb, nnzb, S.n_levels_l(), tt, FC.size(), fs.size(), bs.size(), tasks, hazards_intra, g_fail);
  return g_fail ? 1 : 0;
}
