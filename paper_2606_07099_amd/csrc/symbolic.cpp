// One-time symbolic analysis (host C++); see symbolic.h.
#include "symbolic.h"

#include <algorithm>
#include <complex>
#include <numeric>
#include <queue>

#include "sable_pf.h"

namespace sable {

namespace {

// sorted-vector set union of a and b, dropping `skip1` and `skip2`
void merge_into(std::vector<int32_t>& a, const std::vector<int32_t>& b, int32_t skip1,
                int32_t skip2, std::vector<int32_t>& tmp) {
  tmp.clear();
  size_t i = 0, j = 0;
  while (i < a.size() || j < b.size()) {
    int32_t v;
    if (j >= b.size() || (i < a.size() && a[i] < b[j])) {
      v = a[i++];
    } else if (i >= a.size() || b[j] < a[i]) {
      v = b[j++];
    } else {
      v = a[i];
      ++i;
      ++j;
    }
    if (v != skip1 && v != skip2) tmp.push_back(v);
  }
  a.swap(tmp);
}

int32_t find_sorted(const int32_t* first, const int32_t* last, int32_t key) {
  const int32_t* it = std::lower_bound(first, last, key);
  return (it != last && *it == key) ? (int32_t)(it - first) : -1;
}

}  // namespace

int build_level_chunks(const Symbolic& S, int32_t budget_ints, LevelChunks& out, std::string& err) {
  out = LevelChunks{};
  // generic chunker: items of one level are appended to the current chunk
  // while it fits; emit() closes a chunk
  struct Builder {
    std::vector<int32_t>* ptr;
    std::vector<int32_t>* blob;
    int32_t max_ints = 0;
    std::vector<int32_t> rec, rec2, tail;   // first and second record lists, payload
    int32_t n1 = 0, n2 = 0;
    void emit(const int32_t* hdr4, int32_t end1, int32_t end2) {
      if (n1 == 0) return;
      std::vector<int32_t> c(hdr4, hdr4 + 4);
      c.insert(c.end(), rec.begin(), rec.end());
      c.insert(c.end(), {0, 0, 0, end1});
      if (!rec2.empty() || end2 >= 0) {
        c.insert(c.end(), rec2.begin(), rec2.end());
        c.insert(c.end(), {0, 0, 0, end2});
      }
      c.insert(c.end(), tail.begin(), tail.end());
      while (c.size() % 4) c.push_back(0);
      ptr->push_back((int32_t)blob->size());
      blob->insert(blob->end(), c.begin(), c.end());
      max_ints = std::max<int32_t>(max_ints, (int32_t)c.size());
      rec.clear(); rec2.clear(); tail.clear(); n1 = n2 = 0;
    }
  };
  const int32_t nb = S.nb, tb = S.tail_base;
  // ---- factor
  {
    Builder B{&out.f_ptr, &out.f_blob};
    for (int32_t h = 0; h < S.n_task_levels; ++h) {
      for (int32_t ti = S.task_ptr[h]; ti < S.task_ptr[h + 1]; ++ti) {
        const int32_t a = S.task4[4 * ti], sb = S.task4[4 * ti + 1], se = S.task4[4 * ti + 2];
        const int32_t fin = S.task4[4 * ti + 3];
        int32_t nt = 0;
        for (int32_t i = sb; i < se; ++i) nt += S.step4[4 * i + 3];
        const int32_t need = 4 + 4 * (B.n1 + 2) + 4 * (B.n2 + (se - sb) + 1) + (int32_t)B.tail.size() + nt + 3;
        if (need > budget_ints && B.n1 > 0) {
          const int32_t hdr[4] = {B.n1, B.n2, (int32_t)B.tail.size(), 0};
          B.emit(hdr, B.n2, (int32_t)B.tail.size());
        }
        if (4 + 8 + 4 * ((se - sb) + 1) + nt + 3 > budget_ints) {
          err = "template: a factor task exceeds the metadata chunk budget";
          return -1;
        }
        B.rec.insert(B.rec.end(), {a, S.rp[a], fin ? S.diag[a] - S.rp[a] : -1, B.n2});
        for (int32_t i = sb; i < se; ++i) {
          const int32_t n = S.step4[4 * i + 3], ts = S.step_ts[i];
          B.rec2.insert(B.rec2.end(), {S.step4[4 * i], S.step4[4 * i + 1], S.step4[4 * i + 2],
                                       (int32_t)B.tail.size()});
          for (int32_t t = 0; t < n; ++t) B.tail.push_back(S.upd_tgt[ts + t]);
          B.n2++;
        }
        B.n1++;
      }
      const int32_t hdr[4] = {B.n1, B.n2, (int32_t)B.tail.size(), 0};
      B.emit(hdr, B.n2, (int32_t)B.tail.size());
    }
    out.f_ptr.push_back((int32_t)out.f_blob.size());
    out.max_ints = std::max(out.max_ints, B.max_ints);
  }
  // ---- solves: rows of a level with their column lists
  auto solves = [&](const std::vector<int32_t>& lptr, const std::vector<int32_t>& lrows, int32_t nlev,
                    bool lower, bool pairs, std::vector<int32_t>& ptr, std::vector<int32_t>& blob) -> int {
    const int32_t w = pairs ? 2 : 1;
    Builder B{&ptr, &blob};
    for (int32_t h = 0; h < nlev; ++h) {
      for (int32_t ri = lptr[h]; ri < lptr[h + 1]; ++ri) {
        const int32_t a = lrows[ri];
        const int32_t p0 = lower ? S.rp[a] : S.diag[a] + 1;
        const int32_t p1 = lower ? S.diag[a] : S.rp[a + 1];
        const int32_t need = 4 + 4 * (B.n1 + 2) + (int32_t)B.tail.size() + w * (p1 - p0) + 3;
        if (need > budget_ints && B.n1 > 0) {
          const int32_t hdr[4] = {B.n1, (int32_t)B.tail.size() / w, 0, 0};
          B.emit(hdr, (int32_t)B.tail.size() / w, -1);
        }
        if (4 + 8 + w * (p1 - p0) + 3 > budget_ints) {
          err = "template: a solve row exceeds the metadata chunk budget";
          return -1;
        }
        B.rec.insert(B.rec.end(), {a, p0, 0, (int32_t)B.tail.size() / w});
        for (int32_t p = p0; p < p1; ++p) {
          B.tail.push_back(S.ci[p]);
          if (pairs) B.tail.push_back(S.mirror[p]);
        }
        B.n1++;
      }
      const int32_t hdr[4] = {B.n1, (int32_t)B.tail.size() / w, 0, 0};
      B.emit(hdr, (int32_t)B.tail.size() / w, -1);
    }
    ptr.push_back((int32_t)blob.size());
    out.max_ints = std::max(out.max_ints, B.max_ints);
    return 0;
  };
  const int32_t nbs = (int32_t)S.lev_um_ptr.size() - 1;
  if (solves(S.lev_l_ptr, S.lev_l_rows, S.n_fs_levels, true, false, out.fs_ptr, out.fs_blob)) return -1;
  if (solves(S.lev_um_ptr, S.lev_um_rows, nbs, false, false, out.bs_ptr, out.bs_blob)) return -1;
  if (solves(S.lev_l_ptr, S.lev_l_rows, S.n_fs_levels, true, true, out.ut_ptr, out.ut_blob)) return -1;
  if (solves(S.lev_um_ptr, S.lev_um_rows, nbs, false, true, out.lt_ptr, out.lt_blob)) return -1;
  out.tt_ptr.assign(S.tail_t + 1, 0);
  for (int32_t l = 0; l < S.tail_t; ++l) {
    const int32_t a = tb + l;
    for (int32_t p = S.rp[a]; p < S.tail_split[l]; ++p) {
      out.tt_pairs.push_back(S.ci[p]);
      out.tt_pairs.push_back(S.mirror[p]);
    }
    out.tt_ptr[l + 1] = (int32_t)out.tt_pairs.size() / 2;
  }
  (void)nb;
  (void)tb;
  return 0;
}

int ybus_from_branches(int32_t n_bus, int32_t n_branch, const int32_t* f, const int32_t* t,
                       const double* r, const double* x, const double* bc,
                       std::vector<int32_t>& rp, std::vector<int32_t>& ci,
                       std::vector<double>& g, std::vector<double>& b, std::string& err) {
  if (n_bus <= 0 || n_branch < 0 || (n_branch > 0 && (!f || !t || !r || !x || !bc))) {
    err = "ybus_from_branches: bad sizes or null pointers";
    return PF_EINVAL;
  }
  // (row, col) -> accumulated admittance, via sorted triplets
  struct Trip { int32_t i, j; std::complex<double> y; };
  std::vector<Trip> trips;
  trips.reserve((size_t)n_branch * 4 + n_bus);
  for (int32_t k = 0; k < n_branch; ++k) {
    int32_t a = f[k], c = t[k];
    if (a < 0 || a >= n_bus || c < 0 || c >= n_bus || a == c) {
      err = "ybus_from_branches: branch endpoint out of range or self-loop";
      return PF_EINVAL;
    }
    std::complex<double> z(r[k], x[k]);
    if (std::abs(z) == 0.0) {
      err = "ybus_from_branches: zero series impedance";
      return PF_EINVAL;
    }
    std::complex<double> ys = 1.0 / z, ysh(0.0, 0.5 * bc[k]);
    trips.push_back({a, a, ys + ysh});
    trips.push_back({c, c, ys + ysh});
    trips.push_back({a, c, -ys});
    trips.push_back({c, a, -ys});
  }
  for (int32_t i = 0; i < n_bus; ++i) trips.push_back({i, i, 0.0});  // keep every diagonal
  std::stable_sort(trips.begin(), trips.end(), [](const Trip& p, const Trip& q) {
    return p.i != q.i ? p.i < q.i : p.j < q.j;
  });
  rp.assign(n_bus + 1, 0);
  ci.clear(); g.clear(); b.clear();
  for (size_t s = 0; s < trips.size();) {
    size_t e = s;
    std::complex<double> acc = 0.0;
    while (e < trips.size() && trips[e].i == trips[s].i && trips[e].j == trips[s].j) acc += trips[e++].y;
    ci.push_back(trips[s].j);
    g.push_back(acc.real());
    b.push_back(acc.imag());
    rp[trips[s].i + 1]++;
    s = e;
  }
  for (int32_t i = 0; i < n_bus; ++i) rp[i + 1] += rp[i];
  return (int)ci.size();
}

int analyze(int32_t n_bus, const int32_t* bus_type, const int32_t* y_indptr,
            const int32_t* y_indices, const double* y_g, const double* y_b, Symbolic& S,
            std::string& err, int32_t tail_max) {
  if (n_bus < 2 || !bus_type || !y_indptr || !y_indices || !y_g || !y_b) {
    err = "template: need n_bus >= 2 and non-null bus_type / Y_bus arrays";
    return PF_EINVAL;
  }
  S = Symbolic();
  S.n_bus = n_bus;
  S.bus_type.assign(bus_type, bus_type + n_bus);
  int32_t n_slack = 0;
  for (int32_t i = 0; i < n_bus; ++i) {
    int32_t bt = bus_type[i];
    if (bt < 0 || bt > 2) {
      err = "template: bus_type must be 0 (PQ), 1 (PV) or 2 (slack)";
      return PF_EINVAL;
    }
    if (bt == PF_BUS_SLACK) { S.slack = i; ++n_slack; }
    if (bt == PF_BUS_PV) S.n_pv++;
    if (bt == PF_BUS_PQ) S.n_pq++;
  }
  if (n_slack != 1) {
    err = "template: exactly one slack bus is required";
    return PF_ETOPOLOGY;
  }
  // ---- Y_bus intake: validate, sort columns, reject duplicates
  if (y_indptr[0] != 0) { err = "template: y_indptr[0] must be 0"; return PF_EINVAL; }
  for (int32_t i = 0; i < n_bus; ++i)
    if (y_indptr[i + 1] < y_indptr[i]) { err = "template: y_indptr not monotone"; return PF_EINVAL; }
  const int32_t nnzY = y_indptr[n_bus];
  S.y_rp.assign(y_indptr, y_indptr + n_bus + 1);
  S.y_ci.resize(nnzY); S.y_g.resize(nnzY); S.y_b.resize(nnzY);
  {
    std::vector<int32_t> idx;
    for (int32_t i = 0; i < n_bus; ++i) {
      int32_t s = y_indptr[i], e = y_indptr[i + 1];
      idx.resize(e - s);
      std::iota(idx.begin(), idx.end(), s);
      for (int32_t q = s; q < e; ++q)
        if (y_indices[q] < 0 || y_indices[q] >= n_bus) { err = "template: Y_bus column index out of range"; return PF_EINVAL; }
      std::stable_sort(idx.begin(), idx.end(), [&](int32_t p, int32_t q) { return y_indices[p] < y_indices[q]; });
      for (int32_t q = s; q < e; ++q) {
        int32_t src = idx[q - s];
        S.y_ci[q] = y_indices[src];
        S.y_g[q] = y_g[src];
        S.y_b[q] = y_b[src];
        if (q > s && S.y_ci[q] == S.y_ci[q - 1]) { err = "template: duplicate Y_bus entry"; return PF_EINVAL; }
        if (!std::isfinite(S.y_g[q]) || !std::isfinite(S.y_b[q])) { err = "template: non-finite Y_bus value"; return PF_EINVAL; }
      }
    }
  }
  S.y_tr.assign(nnzY, -1);
  for (int32_t i = 0; i < n_bus; ++i)
    for (int32_t q = S.y_rp[i]; q < S.y_rp[i + 1]; ++q) {
      int32_t j = S.y_ci[q];
      int32_t off = find_sorted(&S.y_ci[S.y_rp[j]], &S.y_ci[0] + S.y_rp[j + 1], i);
      S.y_tr[q] = off < 0 ? -1 : S.y_rp[j] + off;
    }
  // ---- connectivity from the slack over the (symmetrised) Y pattern
  std::vector<std::vector<int32_t>> nbr(n_bus);
  for (int32_t i = 0; i < n_bus; ++i)
    for (int32_t q = S.y_rp[i]; q < S.y_rp[i + 1]; ++q) {
      int32_t j = S.y_ci[q];
      if (j != i) { nbr[i].push_back(j); nbr[j].push_back(i); }
    }
  for (auto& v : nbr) { std::sort(v.begin(), v.end()); v.erase(std::unique(v.begin(), v.end()), v.end()); }
  {
    std::vector<char> seen(n_bus, 0);
    std::queue<int32_t> qu;
    qu.push(S.slack); seen[S.slack] = 1;
    int32_t cnt = 1;
    while (!qu.empty()) {
      int32_t u = qu.front(); qu.pop();
      for (int32_t v : nbr[u]) if (!seen[v]) { seen[v] = 1; ++cnt; qu.push(v); }
    }
    if (cnt != n_bus) { err = "template: network is disconnected (or has an isolated bus)"; return PF_ETOPOLOGY; }
  }
  // ---- compact index of the non-slack buses (ascending bus order)
  const int32_t nb = n_bus - 1;
  S.nb = nb;
  std::vector<int32_t> comp(n_bus, -1), comp_bus(nb);
  for (int32_t i = 0, c = 0; i < n_bus; ++i) if (i != S.slack) { comp[i] = c; comp_bus[c] = i; ++c; }
  std::vector<std::vector<int32_t>> adj(nb);
  for (int32_t c = 0; c < nb; ++c)
    for (int32_t j : nbr[comp_bus[c]]) if (j != S.slack) adj[c].push_back(comp[j]);
  // ---- exact minimum degree on the elimination graph (Tinney scheme 2)
  std::vector<int32_t> order; order.reserve(nb);
  std::vector<std::vector<int32_t>> later(nb);
  std::vector<char> done(nb, 0);
  std::vector<int32_t> tmp;
  for (int32_t step = 0; step < nb; ++step) {
    int32_t v = -1;
    size_t best = SIZE_MAX;
    for (int32_t c = 0; c < nb; ++c)
      if (!done[c] && adj[c].size() < best) { best = adj[c].size(); v = c; }
    order.push_back(v);
    done[v] = 1;
    later[v] = adj[v];
    const std::vector<int32_t>& cl = later[v];
    for (int32_t u : cl) merge_into(adj[u], cl, v, u, tmp);
    adj[v].clear();
  }
  // ---- renumber by (elimination-tree level, elimination position): a
  // topological order of the same elimination tree, hence the same fill,
  // with the highest levels (the top separator) last
  {
    std::vector<int32_t> lvl(nb, 0), pos(nb);
    for (int32_t r = 0; r < nb; ++r) pos[order[r]] = r;
    for (int32_t r = 0; r < nb; ++r) {
      const int32_t v = order[r];
      for (int32_t u : later[v]) lvl[u] = std::max(lvl[u], lvl[v] + 1);
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
      return lvl[x] != lvl[y] ? lvl[x] < lvl[y] : pos[x] < pos[y];
    });
  }
  // ---- block rows in elimination order
  std::vector<int32_t> iperm(nb);
  for (int32_t r = 0; r < nb; ++r) iperm[order[r]] = r;
  S.blk_bus.resize(nb);
  S.bus_blk.assign(n_bus, -1);
  for (int32_t r = 0; r < nb; ++r) { S.blk_bus[r] = comp_bus[order[r]]; S.bus_blk[comp_bus[order[r]]] = r; }
  std::vector<std::vector<int32_t>> rows(nb);   // full row pattern (L, diag, U)
  for (int32_t r = 0; r < nb; ++r) {
    rows[r].push_back(r);
    for (int32_t u : later[order[r]]) {
      int32_t s = iperm[u];
      rows[r].push_back(s);     // U(r, s), s > r
      rows[s].push_back(r);     // L(s, r)
    }
  }
  S.rp.assign(nb + 1, 0);
  for (int32_t r = 0; r < nb; ++r) {
    std::sort(rows[r].begin(), rows[r].end());
    S.rp[r + 1] = S.rp[r] + (int32_t)rows[r].size();
    S.max_row_blocks = std::max<int32_t>(S.max_row_blocks, (int32_t)rows[r].size());
  }
  S.ci.resize(S.rp[nb]);
  S.prow.resize(S.rp[nb]);
  S.diag.resize(nb);
  for (int32_t r = 0; r < nb; ++r) {
    std::copy(rows[r].begin(), rows[r].end(), S.ci.begin() + S.rp[r]);
    for (int32_t p = S.rp[r]; p < S.rp[r + 1]; ++p) S.prow[p] = r;
    S.diag[r] = S.rp[r] + find_sorted(rows[r].data(), rows[r].data() + rows[r].size(), r);
  }
  const int32_t nnzb = S.rp[nb];
  // ---- elimination lists
  S.upd_start.assign(nnzb, 0);
  std::vector<int32_t> pos_in_row(nb, -1);
  for (int32_t a = 0; a < nb; ++a) {
    for (int32_t p = S.rp[a]; p < S.rp[a + 1]; ++p) pos_in_row[S.ci[p]] = p - S.rp[a];
    for (int32_t p = S.rp[a]; p < S.diag[a]; ++p) {
      int32_t k = S.ci[p];
      S.upd_start[p] = (int32_t)S.upd_tgt.size();
      for (int32_t q = S.diag[k] + 1; q < S.rp[k + 1]; ++q) {
        int32_t off = pos_in_row[S.ci[q]];
        if (off < 0) { err = "template: internal error, fill pattern not closed"; return PF_EINVAL; }
        S.upd_tgt.push_back(off);
      }
    }
    for (int32_t p = S.rp[a]; p < S.rp[a + 1]; ++p) pos_in_row[S.ci[p]] = -1;
  }
  S.n_upd = (int64_t)S.upd_tgt.size();
  // ---- level schedules
  std::vector<int32_t> lev_l(nb, 0), lev_u(nb, 0);
  int32_t nl = 0, nu = 0;
  for (int32_t a = 0; a < nb; ++a) {
    int32_t lv = 0;
    for (int32_t p = S.rp[a]; p < S.diag[a]; ++p) lv = std::max(lv, lev_l[S.ci[p]] + 1);
    lev_l[a] = lv;
    nl = std::max(nl, lv + 1);
  }
  for (int32_t a = nb - 1; a >= 0; --a) {
    int32_t lv = 0;
    for (int32_t p = S.diag[a] + 1; p < S.rp[a + 1]; ++p) lv = std::max(lv, lev_u[S.ci[p]] + 1);
    lev_u[a] = lv;
    nu = std::max(nu, lv + 1);
  }
  auto bucket = [&](const std::vector<int32_t>& lev, int32_t n, std::vector<int32_t>& ptr,
                    std::vector<int32_t>& rws) {
    ptr.assign(n + 1, 0);
    for (int32_t a = 0; a < nb; ++a) ptr[lev[a] + 1]++;
    for (int32_t l = 0; l < n; ++l) ptr[l + 1] += ptr[l];
    rws.resize(nb);
    std::vector<int32_t> fillp(ptr.begin(), ptr.end() - 1);
    for (int32_t a = 0; a < nb; ++a) rws[fillp[lev[a]]++] = a;
  };
  bucket(lev_l, nl, S.lev_l_ptr, S.lev_l_rows);
  bucket(lev_u, nu, S.lev_u_ptr, S.lev_u_rows);
  // ---- transposed positions and the Jacobian fill map
  S.mirror.resize(nnzb);
  S.lu_src.assign(nnzb, -1);
  for (int32_t a = 0; a < nb; ++a)
    for (int32_t p = S.rp[a]; p < S.rp[a + 1]; ++p) {
      int32_t j = S.ci[p];
      int32_t off = find_sorted(&S.ci[S.rp[j]], &S.ci[0] + S.rp[j + 1], a);
      S.mirror[p] = S.rp[j] + off;
      int32_t bi = S.blk_bus[a], bj = S.blk_bus[j];
      int32_t yo = find_sorted(&S.y_ci[S.y_rp[bi]], &S.y_ci[0] + S.y_rp[bi + 1], bj);
      S.lu_src[p] = yo < 0 ? -1 : S.y_rp[bi] + yo;
    }
  // ---- dense tail: the rows of the highest levels, at most tail_max of them
  {
    std::vector<int32_t> cnt(nl + 1, 0);
    for (int32_t a = 0; a < nb; ++a) cnt[lev_l[a]]++;
    int32_t h = nl, t = 0;
    while (h > 0 && t + cnt[h - 1] <= std::min<int32_t>(tail_max, 64)) { t += cnt[h - 1]; --h; }
    if (t < 4) { t = 0; h = nl; }
    S.tail_t = t;
    S.tail_h = h;
    S.tail_base = nb - t;
    for (int32_t a = 0; a < nb; ++a)
      if ((a >= S.tail_base) != (lev_l[a] >= h)) { err = "template: internal error, tail rows not last"; return PF_EINVAL; }
    S.tail_pos.assign((size_t)t * t, -1);
    S.tail_split.assign(t, 0);
    for (int32_t i = 0; i < t; ++i) {
      const int32_t a = S.tail_base + i;
      S.tail_split[i] = S.rp[a];
      for (int32_t p = S.rp[a]; p < S.rp[a + 1]; ++p) {
        if (S.ci[p] < S.tail_base) { S.tail_split[i] = p + 1; continue; }
        S.tail_pos[(size_t)i * t + (S.ci[p] - S.tail_base)] = p;
      }
    }
    S.tail_cblk.clear();
    S.tail_lbase.assign(t, 0);
    S.tail_cpos.assign((size_t)t * t, -1);
    for (int32_t i = 0; i < t; ++i) {
      const int32_t a = S.tail_base + i;
      S.tail_lbase[i] = (int32_t)S.tail_cblk.size() - (S.tail_split[i] - S.rp[a]);
      for (int32_t p = S.tail_split[i]; p < S.rp[a + 1]; ++p) {
        S.tail_cpos[(size_t)i * t + (S.ci[p] - S.tail_base)] = (int32_t)S.tail_cblk.size();
        S.tail_cblk.push_back(p);
      }
    }
    S.tail_mask.assign(t ? t + 2 : 0, 0u);
    if (t > 0 && t <= 32)
      for (int32_t i = 0; i < t; ++i)
        for (int32_t j = 0; j < t; ++j) {
          if (S.tail_pos[(size_t)i * t + j] < 0 || i == j) continue;
          if (j > i) { S.tail_mask[i] |= 1u << j; S.tail_mask[t + 1] |= 1u << j; }
          else S.tail_mask[t] |= 1u << j;
        }
  }
  const int32_t tb = S.tail_base;
  {
    const int32_t t = S.tail_t;
    // rows below each tail pivot with a block in its column, in row order
    std::vector<std::vector<int32_t>> by_piv(t);
    for (int32_t i = 0; i < t; ++i) {
      const int32_t a = tb + i;
      for (int32_t p = S.rp[a]; p < S.diag[a]; ++p)
        if (S.ci[p] >= tb) by_piv[S.ci[p] - tb].push_back(p);
    }
    if (S.tail_cblk.size() >= 2048 || t > 32) { err = "template: dense tail too large"; return PF_EINVAL; }
    auto cidx = [&](int32_t a, int32_t p) { return S.tail_lbase[a - tb] + (p - S.rp[a]); };
    S.tail_prog.assign(8 * (size_t)t, 0);
    for (int32_t k = 0; k < t; ++k) {
      const int32_t ak = tb + k;
      const int32_t nu = S.rp[ak + 1] - S.diag[ak] - 1, ns = (int32_t)by_piv[k].size();
      int32_t* r = &S.tail_prog[8 * k];
      r[0] = cidx(ak, S.diag[ak]);
      r[1] = cidx(ak, S.diag[ak] + 1);
      r[2] = nu | (ns << 16);
      uint32_t lm = 0, um = 0;
      for (int32_t p = S.tail_split[k]; p < S.rp[ak + 1]; ++p) {
        const int32_t j = S.ci[p] - tb;
        if (p < S.diag[ak]) lm |= 1u << j;
        else if (p > S.diag[ak]) um |= 1u << j;
      }
      r[5] = (int32_t)lm;
      r[6] = (int32_t)um;
    }
    for (int32_t k = 0; k < t; ++k) {
      S.tail_prog[8 * k + 3] = (int32_t)S.tail_prog.size();
      for (int32_t p : by_piv[k]) S.tail_prog.push_back(cidx(S.prow[p], p) | ((S.prow[p] - tb) << 16));
    }
    S.tail_prog_prefix = (int32_t)S.tail_prog.size();
    for (int32_t k = 0; k < t; ++k) {
      const int32_t nu = S.tail_prog[8 * k + 2] & 0xffff;
      S.tail_prog[8 * k + 4] = (int32_t)S.tail_prog.size();
      for (int32_t p : by_piv[k]) {
        const int32_t a = S.prow[p];
        for (int32_t j = 0; j < nu; ++j) {
          const int32_t tgt = S.tail_lbase[a - tb] + S.upd_tgt[S.upd_start[p] + j];
          S.tail_prog.push_back(tgt | (cidx(a, p) << 11) | (j << 22));
        }
      }
    }
  }
  // ---- factorisation tasks of the barrier-synchronised part: steps grouped
  // by (row, level of the pivot); pivots inside the tail and the tail's own
  // pivot blocks are left to the dense tail
  S.n_task_levels = S.tail_t ? std::min(S.tail_h + 1, nl) : nl;
  S.n_fs_levels = S.tail_t ? S.tail_h : nl;
  const int32_t ntl = S.n_task_levels;
  S.task_ptr.assign(ntl + 1, 0);
  S.task4.clear();
  S.step4.clear();
  S.step_ts.clear();
  {
    std::vector<std::vector<int32_t>> by_level(nl);   // rows with work at each level
    for (int32_t a = 0; a < nb; ++a) {
      if (S.diag[a] == S.rp[a]) by_level[0].push_back(a);
      for (int32_t p = S.rp[a]; p < S.diag[a]; ++p) {
        const int32_t h = lev_l[S.ci[p]] + 1;
        auto& v = by_level[h];
        if (v.empty() || v.back() != a) v.push_back(a);
      }
    }
    for (int32_t h = 0; h < ntl; ++h) {
      S.task_ptr[h] = (int32_t)(S.task4.size() / 4);
      for (int32_t a : by_level[h]) {
        const int32_t sb = (int32_t)S.step_ts.size();
        for (int32_t p = S.rp[a]; p < S.diag[a]; ++p) {
          const int32_t k = S.ci[p];
          if (lev_l[k] + 1 != h || k >= tb) continue;
          S.step4.push_back(p - S.rp[a]);
          S.step4.push_back(k);
          S.step4.push_back(S.diag[k] + 1);
          S.step4.push_back(S.rp[k + 1] - S.diag[k] - 1);
          S.step_ts.push_back(S.upd_start[p]);
        }
        const int32_t fin = (lev_l[a] == h && a < tb) ? 1 : 0;
        if ((int32_t)S.step_ts.size() == sb && !fin) continue;
        S.task4.push_back(a);
        S.task4.push_back(sb);
        S.task4.push_back((int32_t)S.step_ts.size());
        S.task4.push_back(fin);
      }
    }
    S.task_ptr[ntl] = (int32_t)(S.task4.size() / 4);
  }
  // ---- backward-solve levels of the rows outside the tail
  {
    std::vector<int32_t> lv(nb, 0);
    int32_t nlu = 0;
    for (int32_t a = tb - 1; a >= 0; --a) {
      int32_t x = 0;
      for (int32_t p = S.diag[a] + 1; p < S.rp[a + 1]; ++p)
        if (S.ci[p] < tb) x = std::max(x, lv[S.ci[p]] + 1);
      lv[a] = x;
      nlu = std::max(nlu, x + 1);
    }
    S.lev_um_ptr.assign(nlu + 1, 0);
    for (int32_t a = 0; a < tb; ++a) S.lev_um_ptr[lv[a] + 1]++;
    for (int32_t l = 0; l < nlu; ++l) S.lev_um_ptr[l + 1] += S.lev_um_ptr[l];
    S.lev_um_rows.resize(tb);
    std::vector<int32_t> fp(S.lev_um_ptr.begin(), S.lev_um_ptr.end() - 1);
    for (int32_t a = 0; a < tb; ++a) S.lev_um_rows[fp[lv[a]]++] = a;
  }
  // ---- Jacobian fill records
  S.fill4.resize(4 * (size_t)nnzb);
  for (int32_t p = 0; p < nnzb; ++p) {
    const int32_t a = S.prow[p], j = S.ci[p];
    const int32_t bi = S.blk_bus[a], bj = S.blk_bus[j];
    int32_t fl = (a == j ? 1 : 0) | (bus_type[bi] == PF_BUS_PV ? 2 : 0) | (bus_type[bj] == PF_BUS_PV ? 4 : 0);
    S.fill4[4 * p] = S.lu_src[p];
    S.fill4[4 * p + 1] = bi;
    S.fill4[4 * p + 2] = bj;
    S.fill4[4 * p + 3] = fl;
  }
  // ---- statistics
  auto nun = [&](int32_t bus) { return bus_type[bus] == PF_BUS_PQ ? 2 : 1; };
  S.nnz_j1 = 0;
  for (int32_t i = 0; i < n_bus; ++i) {
    if (i == S.slack) continue;
    for (int32_t q = S.y_rp[i]; q < S.y_rp[i + 1]; ++q)
      if (S.y_ci[q] != S.slack) S.nnz_j1 += nun(i) * nun(S.y_ci[q]);
  }
  S.nnz_lu = 0;
  for (int32_t p = 0; p < nnzb; ++p) S.nnz_lu += nun(S.blk_bus[S.prow[p]]) * nun(S.blk_bus[S.ci[p]]);
  int64_t n_lblk = 0;
  for (int32_t a = 0; a < nb; ++a) n_lblk += S.diag[a] - S.rp[a];
  S.factor_flops = 16.0 * (double)(n_lblk + S.n_upd) + 10.0 * nb;
  return PF_OK;
}

}  // namespace sable
