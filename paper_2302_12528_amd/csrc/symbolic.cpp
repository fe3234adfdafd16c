// Host ordering and symbolic analysis (see symbolic.hpp).
#include "symbolic.hpp"

#include <algorithm>
#include <array>
#include <functional>
#include <numeric>

namespace lobpcg {
namespace {

struct Builder {
  int64_t n;
  const int32_t* rowptr;
  const int32_t* colind;
  int leaf;
  int64_t offset = 0;          // first node of the component being ordered
  std::vector<int32_t> perm;   // filled in emission order
  std::vector<int32_t> begin, nc, parent;
  int32_t next = 0;
  // scratch for graph bisection
  std::vector<int32_t> stamp, lvl;
  int32_t cur_stamp = 0;

  int new_sn(const std::vector<int32_t>& nodes) {
    int s = (int)begin.size();
    begin.push_back(next);
    nc.push_back((int32_t)nodes.size());
    parent.push_back(-1);
    for (int32_t v : nodes) perm[next++] = v;
    return s;
  }

  // Geometric nested dissection of the box [lo, hi) of a g0 x g1 x g2 grid.
  std::vector<int> box(const int g[3], std::array<int, 3> lo, std::array<int, 3> hi) {
    int64_t vol = 1;
    for (int d = 0; d < 3; ++d) vol *= std::max(0, hi[d] - lo[d]);
    if (vol == 0) return {};
    int d = 0;
    for (int e = 1; e < 3; ++e)
      if (hi[e] - lo[e] > hi[d] - lo[d]) d = e;
    if (vol <= leaf || hi[d] - lo[d] < 2) {
      std::vector<int32_t> nodes;
      nodes.reserve(vol);
      for (int i = lo[0]; i < hi[0]; ++i)
        for (int j = lo[1]; j < hi[1]; ++j)
          for (int l = lo[2]; l < hi[2]; ++l) nodes.push_back((int32_t)(offset + ((int64_t)i * g[1] + j) * g[2] + l));
      return {new_sn(nodes)};
    }
    int mid = lo[d] + (hi[d] - lo[d]) / 2;
    auto hl = hi; hl[d] = mid;
    auto lr = lo; lr[d] = mid + 1;
    std::vector<int> a = box(g, lo, hl);
    std::vector<int> b = box(g, lr, hi);
    auto ls = lo; ls[d] = mid;
    auto hs = hi; hs[d] = mid + 1;
    std::vector<int32_t> sep;
    for (int i = ls[0]; i < hs[0]; ++i)
      for (int j = ls[1]; j < hs[1]; ++j)
        for (int l = ls[2]; l < hs[2]; ++l) sep.push_back((int32_t)(offset + ((int64_t)i * g[1] + j) * g[2] + l));
    int s = new_sn(sep);
    for (int c : a) parent[c] = s;
    for (int c : b) parent[c] = s;
    return {s};
  }

  // BFS inside the node set marked with `st`; returns visit order, fills lvl.
  std::vector<int32_t> bfs(int32_t start, int32_t st, int32_t visit_st, int& depth) {
    std::vector<int32_t> order{start};
    stamp[start] = visit_st;
    lvl[start] = 0;
    depth = 0;
    for (size_t h = 0; h < order.size(); ++h) {
      int32_t v = order[h];
      for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        int32_t u = colind[e];
        if (stamp[u] == st) {
          stamp[u] = visit_st;
          lvl[u] = lvl[v] + 1;
          depth = std::max(depth, lvl[u]);
          order.push_back(u);
        }
      }
    }
    return order;
  }

  // Graph nested dissection by breadth-first level structures.
  std::vector<int> graph(std::vector<int32_t> nodes) {
    if (nodes.empty()) return {};
    if ((int64_t)nodes.size() <= leaf) return {new_sn(nodes)};
    int32_t st = ++cur_stamp;
    for (int32_t v : nodes) stamp[v] = st;
    // pseudo-peripheral start: two sweeps
    int depth = 0;
    int32_t vs = ++cur_stamp;
    std::vector<int32_t> order = bfs(nodes[0], st, vs, depth);
    if (order.size() == nodes.size()) {
      int32_t far = order.back();
      int32_t st2 = ++cur_stamp;
      for (int32_t v : nodes) stamp[v] = st2;
      int32_t vs2 = ++cur_stamp;
      order = bfs(far, st2, vs2, depth);
    }
    if (order.size() < nodes.size()) {
      // disconnected: split off the reached component, no separator
      std::vector<int32_t> rest;
      int32_t vis = stamp[order[0]];
      for (int32_t v : nodes)
        if (stamp[v] != vis) rest.push_back(v);
      std::vector<int> a = graph(order);
      std::vector<int> b = graph(rest);
      a.insert(a.end(), b.begin(), b.end());
      return a;
    }
    if (depth < 2) return {new_sn(nodes)};
    std::vector<int64_t> cnt(depth + 1, 0);
    for (int32_t v : order) cnt[lvl[v]]++;
    int64_t half = (int64_t)nodes.size() / 2, acc = 0;
    int cut = 1;
    for (int l = 0; l <= depth; ++l) {
      acc += cnt[l];
      if (acc >= half) { cut = l; break; }
    }
    cut = std::min(std::max(cut, 1), depth - 1);
    std::vector<int32_t> left, sep, right;
    for (int32_t v : order) {
      if (lvl[v] < cut) left.push_back(v);
      else if (lvl[v] == cut) sep.push_back(v);
      else right.push_back(v);
    }
    std::vector<int> a = graph(left);
    std::vector<int> b = graph(right);
    int s = new_sn(sep);
    for (int c : a) parent[c] = s;
    for (int c : b) parent[c] = s;
    return {s};
  }
};

}  // namespace

std::string analyze(int64_t n, const int32_t* rowptr, const int32_t* colind, const int32_t grid[3],
                    bool dense, int leaf_size, Symbolic& S) {
  Component c;
  c.off = 0;
  c.n = n;
  for (int d = 0; d < 3; ++d) c.grid[d] = grid ? grid[d] : 0;
  return analyze_multi(n, rowptr, colind, std::vector<Component>{c}, dense, leaf_size, S);
}

std::string analyze_multi(int64_t n, const int32_t* rowptr, const int32_t* colind, const std::vector<Component>& comps,
                          bool dense, int leaf_size, Symbolic& S) {
  if (n <= 0) return "n must be positive";
  Builder B;
  B.n = n;
  B.rowptr = rowptr;
  B.colind = colind;
  B.leaf = leaf_size >= 1 ? leaf_size : 64;
  B.perm.assign(n, -1);
  if (dense) {
    if (comps.size() != 1) return "dense matrices are not batched";
    std::vector<int32_t> all(n);
    std::iota(all.begin(), all.end(), 0);
    B.new_sn(all);
  } else {
    int64_t expect = 0;
    for (const Component& c : comps) {
      if (c.off != expect || c.n <= 0) return "components must tile the index range in order";
      expect += c.n;
      const bool use_grid = c.grid[0] > 0 && c.grid[1] > 0 && c.grid[2] > 0 &&
                            (int64_t)c.grid[0] * c.grid[1] * c.grid[2] == c.n;
      B.offset = c.off;
      if (leaf_size < 1) B.leaf = default_leaf(use_grid ? c.grid : nullptr);
      if (use_grid) {
        int g[3] = {c.grid[0], c.grid[1], c.grid[2]};
        B.box(g, {0, 0, 0}, {g[0], g[1], g[2]});
      } else {
        if (B.stamp.empty()) {
          B.stamp.assign(n, 0);
          B.lvl.assign(n, 0);
        }
        std::vector<int32_t> nodes(c.n);
        std::iota(nodes.begin(), nodes.end(), (int32_t)c.off);
        B.graph(nodes);
      }
      if (B.next != c.off + c.n) return "component ordering leaked outside its index range";
    }
    if (expect != n) return "components do not cover all nodes";
  }
  if (B.next != n) return "ordering did not cover all nodes";
  S = Symbolic();
  S.n = n;
  S.perm = std::move(B.perm);
  S.iperm.assign(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    int32_t o = S.perm[i];
    if (o < 0 || o >= n || S.iperm[o] != -1) return "ordering is not a permutation";
    S.iperm[o] = (int32_t)i;
  }
  const int ns = (int)B.begin.size();
  S.nsuper = ns;
  S.begin = B.begin;
  S.nc = B.nc;
  S.parent = B.parent;
  // children
  S.child_ptr.assign(ns + 1, 0);
  for (int s = 0; s < ns; ++s)
    if (S.parent[s] >= 0) {
      if (S.parent[s] <= s) return "supernode tree not in postorder";
      S.child_ptr[S.parent[s] + 1]++;
    }
  for (int s = 0; s < ns; ++s) S.child_ptr[s + 1] += S.child_ptr[s];
  S.child_list.assign(S.child_ptr[ns], 0);
  {
    std::vector<int32_t> fill(S.child_ptr.begin(), S.child_ptr.end() - 1);
    for (int s = 0; s < ns; ++s)
      if (S.parent[s] >= 0) S.child_list[fill[S.parent[s]]++] = s;
  }
  // row structure
  S.nr.assign(ns, 0);
  S.row_off.assign(ns + 1, 0);
  std::vector<int32_t> mark(n, -1);
  std::vector<std::vector<int32_t>> below(ns);
  for (int s = 0; s < ns; ++s) {
    const int32_t b = S.begin[s], e = S.begin[s] + S.nc[s];
    std::vector<int32_t>& st = below[s];
    if (!dense) {
      for (int32_t j = b; j < e; ++j) {
        int32_t o = S.perm[j];
        for (int32_t q = rowptr[o]; q < rowptr[o + 1]; ++q) {
          int32_t u = S.iperm[colind[q]];
          if (u >= e && mark[u] != s) { mark[u] = s; st.push_back(u); }
        }
      }
    }
    for (int32_t q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
      int c = S.child_list[q];
      for (int32_t r : below[c]) {
        if (r < b) return "child row structure outside parent (invalid ordering)";
        if (r >= e && mark[r] != s) { mark[r] = s; st.push_back(r); }
      }
    }
    std::sort(st.begin(), st.end());
    S.nr[s] = S.nc[s] + (int32_t)st.size();
  }
  for (int s = 0; s < ns; ++s) S.row_off[s + 1] = S.row_off[s] + S.nr[s];
  S.rows.assign(S.row_off[ns], 0);
  S.relpos.assign(S.row_off[ns], -1);
  for (int s = 0; s < ns; ++s) {
    int64_t o = S.row_off[s];
    for (int t = 0; t < S.nc[s]; ++t) S.rows[o + t] = S.begin[s] + t;
    for (size_t j = 0; j < below[s].size(); ++j) S.rows[o + S.nc[s] + j] = below[s][j];
  }
  // relative positions of each child's below rows in its parent's rows, and inverse maps
  S.inv_off.assign(ns + 1, 0);
  for (int s = 0; s < ns; ++s) S.inv_off[s + 1] = S.inv_off[s] + (S.parent[s] >= 0 ? S.nr[S.parent[s]] : 0);
  S.invmap.assign(S.inv_off[ns], -1);
  for (int c = 0; c < ns; ++c) {
    int p = S.parent[c];
    if (p < 0) {
      if (S.nr[c] != S.nc[c]) return "root supernode has rows below it";
      continue;
    }
    const int32_t* prow = &S.rows[S.row_off[p]];
    int pnr = S.nr[p], pnc = S.nc[p];
    for (int j = 0; j < S.nr[c] - S.nc[c]; ++j) {
      int32_t r = S.rows[S.row_off[c] + S.nc[c] + j];
      int pos;
      if (r < S.begin[p] + pnc) {
        pos = r - S.begin[p];
      } else {
        const int32_t* it = std::lower_bound(prow + pnc, prow + pnr, r);
        if (it == prow + pnr || *it != r) return "child row missing from parent structure";
        pos = (int)(it - prow);
      }
      S.relpos[S.row_off[c] + S.nc[c] + j] = pos;
      S.invmap[S.inv_off[c] + pos] = j;
    }
  }
  // levels
  S.level.assign(ns, 0);
  int maxl = 0;
  for (int s = 0; s < ns; ++s) {
    int l = 0;
    for (int32_t q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) l = std::max(l, S.level[S.child_list[q]] + 1);
    S.level[s] = l;
    maxl = std::max(maxl, l);
  }
  S.nlevels = maxl + 1;
  S.level_ptr.assign(S.nlevels + 1, 0);
  for (int s = 0; s < ns; ++s) S.level_ptr[S.level[s] + 1]++;
  for (int l = 0; l < S.nlevels; ++l) S.level_ptr[l + 1] += S.level_ptr[l];
  S.level_sn.assign(ns, 0);
  {
    std::vector<int32_t> fill(S.level_ptr.begin(), S.level_ptr.end() - 1);
    for (int s = 0; s < ns; ++s) S.level_sn[fill[S.level[s]]++] = s;
  }
  // storage plans
  S.panel_off.assign(ns + 1, 0);
  S.upd_off.assign(ns + 1, 0);
  S.uvec_off.assign(ns + 1, 0);
  S.dinv_off.assign(ns + 1, 0);
  S.lcopy_off.assign(ns, 0);
  S.nnz_lower = 0;
  S.flops = 0;
  for (int s = 0; s < ns; ++s) {
    int64_t r = S.nr[s], c = S.nc[s], b = r - c;
    int64_t np = (c + kTile - 1) / kTile;
    S.panel_off[s + 1] = S.panel_off[s] + panel_ld(r) * c;
    S.upd_off[s + 1] = S.upd_off[s] + b * b;
    S.uvec_off[s + 1] = S.uvec_off[s] + b;
    S.dinv_off[s + 1] = S.dinv_off[s] + 2 * np * kTile * kTile;   // inv(L_pp) tiles, then L_pp tiles
    S.nnz_lower += (double)c * (c + 1) / 2 + (double)b * c;
    for (int64_t j = 0; j < c; ++j) {
      double cj = (double)(r - j - 1);
      S.flops += cj * cj + cj;   // column scaling + rank-1 update of the trailing front
    }
    S.max_nr = std::max<int32_t>(S.max_nr, (int32_t)r);
    S.max_nc = std::max<int32_t>(S.max_nc, (int32_t)c);
  }
  S.panel_total = S.panel_off[ns];
  S.upd_total = S.upd_off[ns];
  S.uvec_total = S.uvec_off[ns];
  S.dinv_total = S.dinv_off[ns];
  S.lcopy_max = 0;
  for (int l = 0; l < S.nlevels; ++l) {
    int64_t acc = 0;
    for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
      int s = S.level_sn[q];
      S.lcopy_off[s] = acc;   // L11 copy (nc x nc), inversion scratch (nc x nc), L21 copy (nb x nc)
      acc += 2 * (int64_t)S.nc[s] * S.nc[s] + (int64_t)(S.nr[s] - S.nc[s]) * S.nc[s];
    }
    S.lcopy_max = std::max(S.lcopy_max, acc);
  }
  return "";
}

void permute_pattern(const Symbolic& S, const int32_t* rowptr, const int32_t* colind,
                     std::vector<int32_t>& prow, std::vector<int32_t>& pcol, std::vector<int32_t>& map) {
  const int64_t n = S.n;
  prow.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int32_t o = S.perm[i];
    prow[i + 1] = prow[i] + (rowptr[o + 1] - rowptr[o]);
  }
  pcol.assign(prow[n], 0);
  map.assign(prow[n], 0);
  std::vector<std::pair<int32_t, int32_t>> tmp;
  for (int64_t i = 0; i < n; ++i) {
    int32_t o = S.perm[i];
    tmp.clear();
    for (int32_t e = rowptr[o]; e < rowptr[o + 1]; ++e) tmp.emplace_back(S.iperm[colind[e]], e);
    std::sort(tmp.begin(), tmp.end());
    for (size_t q = 0; q < tmp.size(); ++q) {
      pcol[prow[i] + q] = tmp[q].first;
      map[prow[i] + q] = tmp[q].second;
    }
  }
}

void assembly_positions(const Symbolic& S, const std::vector<int32_t>& prow,
                        const std::vector<int32_t>& pcol, std::vector<int32_t>& apos) {
  const int64_t n = S.n;
  std::vector<int32_t> sn_of(n);
  for (int s = 0; s < S.nsuper; ++s)
    for (int t = 0; t < S.nc[s]; ++t) sn_of[S.begin[s] + t] = s;
  apos.assign(prow[n], -1);
  for (int64_t j = 0; j < n; ++j) {
    int s = sn_of[j];
    const int32_t* r0 = &S.rows[S.row_off[s]];
    const int32_t* r1 = r0 + S.nr[s];
    for (int32_t e = prow[j]; e < prow[j + 1]; ++e) {
      int32_t i = pcol[e];
      if (i < j) continue;
      int pos;
      if (i < S.begin[s] + S.nc[s]) {
        pos = i - S.begin[s];
      } else {
        const int32_t* it = std::lower_bound(r0 + S.nc[s], r1, i);
        pos = (it != r1 && *it == i) ? (int)(it - r0) : -1;
      }
      apos[e] = pos;
    }
  }
}

int64_t exact_fill(int64_t n, const std::vector<int32_t>& prow, const std::vector<int32_t>& pcol) {
  // elimination tree of the lower triangle (ancestors with path compression)
  std::vector<int32_t> parent(n, -1), anc(n, -1);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t e = prow[i]; e < prow[i + 1]; ++e) {
      int32_t k = pcol[e];
      while (k >= 0 && k < i) {
        const int32_t next = anc[k];
        anc[k] = (int32_t)i;
        if (next < 0) {
          parent[k] = (int32_t)i;
          break;
        }
        k = next;
      }
    }
  // row i of L: the union of the tree paths from each k < i with A(i, k) != 0 up to i
  std::vector<int32_t> mark(n, -1);
  int64_t count = n;
  for (int64_t i = 0; i < n; ++i) {
    mark[i] = (int32_t)i;
    for (int32_t e = prow[i]; e < prow[i + 1]; ++e)
      for (int32_t k = pcol[e]; k >= 0 && k < i && mark[k] != i; k = parent[k]) {
        mark[k] = (int32_t)i;
        ++count;
      }
  }
  return count;
}

void build_factor_plan(const Symbolic& S, FactorPlan& P, int schur_wide_tiles) {
  P = FactorPlan();
  P.schur_wide_tiles = std::max(1, schur_wide_tiles);
  const int wide = P.schur_wide_tiles;
  auto push = [&](int s, int I, int J, int p) {
    P.tasks.push_back(s); P.tasks.push_back(I); P.tasks.push_back(J); P.tasks.push_back(p);
  };
  auto ntiles = [](int x) { return (x + kTile - 1) / kTile; };
  P.asm_level_off.assign(S.nlevels + 1, 0);
  for (int l = 0; l < S.nlevels; ++l) {
    const int32_t q0 = S.level_ptr[l], q1 = S.level_ptr[l + 1];
    for (int32_t q = q0; q < q1; ++q) {
      int s = S.level_sn[q];
      for (int t = 0; t < S.nr[s]; ++t) { P.asm_items.push_back(s); P.asm_items.push_back(t); }
    }
    P.asm_level_off[l + 1] = (int64_t)P.asm_items.size() / 2;
    int lmax = 0;
    for (int32_t q = q0; q < q1; ++q) lmax = std::max(lmax, S.nr[S.level_sn[q]]);
    P.level_max_nr.push_back(lmax);
    int maxnp = 0;
    for (int32_t q = q0; q < q1; ++q) maxnp = std::max(maxnp, ntiles(S.nc[S.level_sn[q]]));
    auto begin_step = [&](int kind) {
      FactorPlan::Step st;
      st.off = (int64_t)P.tasks.size() / 4;
      st.count = 0;
      st.kind = kind;
      st.level = l;
      P.steps.push_back(st);
    };
    auto end_step = [&]() {
      FactorPlan::Step& st = P.steps.back();
      st.count = (int32_t)((int64_t)P.tasks.size() / 4 - st.off);
      if (st.count == 0) P.steps.pop_back();
    };
    begin_step(kAssemble);
    push(l, 0, 0, 0);   // one marker task: the assembly kernel reads asm_items of level l
    end_step();
    for (int p = 0; p < maxnp; ++p) {
      // diagonal tile p and the tiles below it in one step: every task first applies panel p - 1 to
      // its tile; task (s, p, p, p) writes L_pp and its inverse, tasks (s, I > p, p, p) the trsm of
      // tile (I, p)
      begin_step(kPotrf);
      for (int32_t q = q0; q < q1; ++q) {
        int s = S.level_sn[q];
        int np = ntiles(S.nc[s]), rt = np + ntiles(S.nr[s] - S.nc[s]);
        if (np > p)
          for (int I = p; I < rt; ++I) push(s, I, p, p);
      }
      end_step();
      // trailing update of the panel columns beyond p + 1 (column p + 1 is updated by the next panel
      // step's own tasks, so that step needs no launch of its own before it: one step of lookahead);
      // task (s, p, p, p) moves L_pp from its staging slot into the panel (the panel step's other
      // tasks read the unfactored tile (p, p) while it is formed)
      begin_step(kUpdate);
      for (int32_t q = q0; q < q1; ++q) {
        int s = S.level_sn[q];
        int np = ntiles(S.nc[s]), rt = np + ntiles(S.nr[s] - S.nc[s]);
        if (np > p) push(s, p, p, p);
        for (int J = p + 2; J < np; ++J)
          for (int I = J; I < rt; ++I) push(s, I, J, p);
      }
      end_step();
    }
    // Schur complement U_s -= L21 L21^T, once, with the whole reduction range nc per tile
    begin_step(kSchur);
    for (int32_t q = q0; q < q1; ++q) {
      int s = S.level_sn[q];
      int np = ntiles(S.nc[s]), rt = np + ntiles(S.nr[s] - S.nc[s]);
      if (rt - np >= wide) continue;
      for (int J = np; J < rt; ++J)
        for (int I = J; I < rt; ++I) push(s, I, J, 0);
    }
    end_step();
    begin_step(kSchur2);
    for (int32_t q = q0; q < q1; ++q) {
      int s = S.level_sn[q];
      int np = ntiles(S.nc[s]), rt = np + ntiles(S.nr[s] - S.nc[s]);
      if (rt - np < wide) continue;
      for (int J = np; J < rt; J += 2)
        for (int I = J; I < rt; I += 2) push(s, I, J, 0);
    }
    end_step();
    // inverse phase: P_s = [inv(L11); L21 inv(L11)].  X = inv(L11) by recursive doubling over
    // diagonal blocks of 2^t tiles: with a block split into halves [[A, 0], [B, C]] whose inverses
    // are known, the lower-left block of its inverse is -inv(C) (B inv(A)); level t forms
    // T1 = B inv(A) (kInvT1) and then -inv(C) T1 (kInvX21) for every block at once.  Finally the
    // rows below: L21 X (kInvP21), from a copy of L21.
    begin_step(kInvPrep);
    for (int32_t q = q0; q < q1; ++q) {
      int s = S.level_sn[q];
      for (int t = 0; t < S.nc[s]; ++t) push(s, t, 0, 0);
    }
    end_step();
    for (int t = 1; (1 << (t - 1)) < maxnp; ++t) {
      for (int kind : {kInvT1, kInvX21}) {
        begin_step(kind);
        for (int32_t q = q0; q < q1; ++q) {
          int s = S.level_sn[q];
          int np = ntiles(S.nc[s]);
          for (int j0 = 0; j0 < np; j0 += (1 << t)) {
            const int m = j0 + (1 << (t - 1));
            const int i1 = std::min(np, j0 + (1 << t));
            for (int I = m; I < i1; ++I)
              for (int J = j0; J < m; ++J) push(s, I, J, t);
          }
        }
        end_step();
      }
    }
    begin_step(kInvP21);
    for (int32_t q = q0; q < q1; ++q) {
      int s = S.level_sn[q];
      int np = ntiles(S.nc[s]), rt = np + ntiles(S.nr[s] - S.nc[s]);
      for (int I = np; I < rt; ++I)
        for (int J = 0; J < np; ++J) push(s, I, J, 0);
    }
    end_step();
  }
}

namespace {

// Item metadata shared by the per-level and the subtree lists (see SolvePlan).
void push_item(const Symbolic& S, const SolvePlan& P, std::vector<int32_t>& items, int s, int t, int k0, int k1,
               int slot, bool fwd) {
  const int64_t po = S.panel_off[s];
  items.insert(items.end(), {s, t, k0, k1, slot, S.begin[s], S.nr[s], S.nc[s], (int32_t)(po & 0xffffffff),
                             (int32_t)(po >> 32), (int32_t)(fwd ? S.uvec_off[s] : P.bwd_src_off[s]),
                             (int32_t)(S.child_ptr[s + 1] > S.child_ptr[s] ? 1 : 0)});
}

// Gather rows of supernode s (with children): own rows somebody contributes to, and every below row.
void push_gather(const Symbolic& S, std::vector<int32_t>& dst, std::vector<int32_t>& ptr, std::vector<int32_t>& src,
                 int s) {
  const int nc = S.nc[s], nr = S.nr[s];
  if (S.child_ptr[s + 1] == S.child_ptr[s]) return;
  for (int r = 0; r < nr; ++r) {
    const size_t before = src.size();
    for (int32_t cq = S.child_ptr[s]; cq < S.child_ptr[s + 1]; ++cq) {
      const int c = S.child_list[cq];
      const int32_t jr = S.invmap[S.inv_off[c] + r];
      if (jr >= 0) src.push_back((int32_t)(S.uvec_off[c] + jr));
    }
    if (r < nc && src.size() == before) continue;   // own row nobody contributes to
    dst.push_back(r < nc ? S.begin[s] + r : -(int32_t)(S.uvec_off[s] + r - nc) - 1);
    ptr.push_back((int32_t)src.size());
  }
}

void build_subtree_lists(const Symbolic& S, int rpt, int sub_levels, SolvePlan& P) {
  const int ns = S.nsuper;
  auto roots_for = [&](int L, std::vector<int>& roots) {
    roots.clear();
    for (int s = 0; s < ns; ++s)
      if (S.level[s] < L && (S.parent[s] < 0 || S.level[S.parent[s]] >= L)) roots.push_back(s);
  };
  std::vector<int> roots;
  if (sub_levels < 0) {
    // the whole tree when its panels are small: its levels are then launch-latency bound.  Larger
    // trees keep one launch per level: a level's tiles spread over the whole chip finish sooner
    // than a subtree's levels run one after another inside a workgroup (measured on the 64^3
    // diffusion problem for cuts of 1 to 4 levels).
    double bytes = 0;
    for (int s = 0; s < ns; ++s) bytes += (double)S.nr[s] * S.nc[s] * 4;
    sub_levels = (bytes <= 4e6) ? S.nlevels : 0;
  }
  sub_levels = std::max(0, std::min(sub_levels, S.nlevels));
  P.sub_levels = sub_levels;
  P.nsub = 0;
  P.sub_gather_ptr.assign(1, 0);
  if (sub_levels == 0) return;
  roots_for(sub_levels, roots);
  P.nsub = (int64_t)roots.size();
  const int L = sub_levels;
  P.sub_gather_off.assign(P.nsub * L + 1, 0);
  P.sub_fwd_off.assign(P.nsub * L + 1, 0);
  P.sub_bwd_off.assign(P.nsub * L + 1, 0);
  std::vector<std::vector<int>> by_level(L);
  std::vector<int> stack;
  for (int64_t q = 0; q < P.nsub; ++q) {
    for (auto& v : by_level) v.clear();
    stack.assign(1, roots[q]);
    while (!stack.empty()) {
      const int s = stack.back();
      stack.pop_back();
      by_level[S.level[s]].push_back(s);
      for (int32_t cq = S.child_ptr[s]; cq < S.child_ptr[s + 1]; ++cq) stack.push_back(S.child_list[cq]);
    }
    for (int l = 0; l < L; ++l) {
      std::sort(by_level[l].begin(), by_level[l].end());
      const int64_t e = q * L + l;
      for (int s : by_level[l]) push_gather(S, P.sub_gather_dst, P.sub_gather_ptr, P.sub_gather_src, s);
      P.sub_gather_off[e + 1] = (int64_t)P.sub_gather_dst.size();
      for (int s : by_level[l])
        for (int t = 0; t < (S.nr[s] + rpt - 1) / rpt; ++t) {
          const int r0 = t * rpt;
          push_item(S, P, P.sub_fwd_items, s, t, 0, (r0 < S.nc[s]) ? std::min(S.nc[s], r0 + rpt) : S.nc[s], -1, true);
        }
      P.sub_fwd_off[e + 1] = (int64_t)P.sub_fwd_items.size() / kSolveItemInts;
      for (int s : by_level[l])
        for (int t = 0; t < (S.nc[s] + rpt - 1) / rpt; ++t) push_item(S, P, P.sub_bwd_items, s, t, t * rpt, S.nr[s], -1, false);
      P.sub_bwd_off[e + 1] = (int64_t)P.sub_bwd_items.size() / kSolveItemInts;
    }
  }
}

}  // namespace

void build_solve_plan(const Symbolic& S, int rpt, int split_target, SolvePlan& P, int sub_levels) {
  P = SolvePlan();
  P.rows_per_tile = rpt;
  P.split_target = split_target;
  P.gather_level_off.assign(S.nlevels + 1, 0);
  P.fwd_level_off.assign(S.nlevels + 1, 0);
  P.bwd_level_off.assign(S.nlevels + 1, 0);
  P.fwd_fin_level_off.assign(S.nlevels + 1, 0);
  P.bwd_fin_level_off.assign(S.nlevels + 1, 0);
  P.gather_ptr.push_back(0);
  P.bwd_src_off.assign(S.nsuper, 0);
  for (int s = 0; s < S.nsuper; ++s) {
    P.bwd_src_off[s] = (int64_t)P.bwd_src.size();
    const int nc = S.nc[s], nr = S.nr[s];
    for (int k = 0; k < nr; ++k)
      P.bwd_src.push_back(k < nc ? S.begin[s] + k : (int32_t)(S.n + S.rows[S.row_off[s] + k]));
    P.bwd_src.resize((size_t)(P.bwd_src_off[s] + panel_ld(nr)), 0);
  }
  // chunks of the reduction range [k0, k1) for a tile, nch wanted
  int maxk = 0;   // longest reduction range of the level being built
  auto emit = [&](std::vector<int32_t>& items, std::vector<int32_t>& fin, int64_t& slots, int s, int t, int k0,
                  int k1, int nch, bool fwd) {
    const int len = k1 - k0;
    int chunk = (len + nch - 1) / nch;
    chunk = std::max(64, (chunk + 15) / 16 * 16);
    nch = (len + chunk - 1) / chunk;
    const int64_t po = S.panel_off[s];
    const int32_t meta[7] = {S.begin[s], S.nr[s], S.nc[s], (int32_t)(po & 0xffffffff), (int32_t)(po >> 32),
                             (int32_t)(fwd ? S.uvec_off[s] : P.bwd_src_off[s]),
                             (int32_t)(S.child_ptr[s + 1] > S.child_ptr[s] ? 1 : 0)};
    auto push = [&](int a, int b, int slot) {
      items.insert(items.end(), {s, t, a, b, slot});
      items.insert(items.end(), meta, meta + 7);
      maxk = std::max(maxk, b - a);
    };
    if (nch <= 1) {
      push(k0, k1, -1);
      return;
    }
    fin.insert(fin.end(), {s, t, (int32_t)slots, nch});
    for (int q = 0; q < nch; ++q) {
      const int a = k0 + q * chunk, b = std::min(k1, a + chunk);
      push(a, b, (int32_t)(slots + q));
    }
    slots += nch;
  };
  for (int l = 0; l < S.nlevels; ++l) {
    int64_t ftiles = 0, btiles = 0;
    for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
      const int s = S.level_sn[q];
      ftiles += (S.nr[s] + rpt - 1) / rpt;
      btiles += (S.nc[s] + rpt - 1) / rpt;
    }
    const int fsplit = (int)std::max<int64_t>(1, split_target / std::max<int64_t>(1, ftiles));
    const int bsplit = (int)std::max<int64_t>(1, split_target / std::max<int64_t>(1, btiles));
    for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
      const int s = S.level_sn[q];
      const int nc = S.nc[s], nr = S.nr[s];
      if (S.child_ptr[s + 1] > S.child_ptr[s]) {
        for (int r = 0; r < nr; ++r) {
          const size_t before = P.gather_src.size();
          for (int32_t cq = S.child_ptr[s]; cq < S.child_ptr[s + 1]; ++cq) {
            const int c = S.child_list[cq];
            const int32_t jr = S.invmap[S.inv_off[c] + r];
            if (jr >= 0) P.gather_src.push_back((int32_t)(S.uvec_off[c] + jr));
          }
          if (r < nc && P.gather_src.size() == before) continue;   // own row nobody contributes to
          P.gather_dst.push_back(r < nc ? S.begin[s] + r : -(int32_t)(S.uvec_off[s] + r - nc) - 1);
          P.gather_ptr.push_back((int32_t)P.gather_src.size());
        }
      }
    }
    maxk = 0;
    for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
      const int s = S.level_sn[q];
      const int nc = S.nc[s], nr = S.nr[s];
      for (int t = 0; t < (nr + rpt - 1) / rpt; ++t) {
        const int r0 = t * rpt;
        const int kmax = (r0 < nc) ? std::min(nc, r0 + rpt) : nc;
        emit(P.fwd_items, P.fwd_fin, P.fwd_slots, s, t, 0, kmax, fsplit, true);
      }
    }
    P.fwd_wide.push_back(maxk > kSolveWideK);
    maxk = 0;
    for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
      const int s = S.level_sn[q];
      const int nc = S.nc[s], nr = S.nr[s];
      for (int t = 0; t < (nc + rpt - 1) / rpt; ++t)
        emit(P.bwd_items, P.bwd_fin, P.bwd_slots, s, t, t * rpt, nr, bsplit, false);
    }
    P.bwd_wide.push_back(maxk > kSolveWideK);
    P.gather_level_off[l + 1] = (int64_t)P.gather_dst.size();
    P.fwd_level_off[l + 1] = (int64_t)P.fwd_items.size() / kSolveItemInts;
    P.bwd_level_off[l + 1] = (int64_t)P.bwd_items.size() / kSolveItemInts;
    P.fwd_fin_level_off[l + 1] = (int64_t)P.fwd_fin.size() / 4;
    P.bwd_fin_level_off[l + 1] = (int64_t)P.bwd_fin.size() / 4;
  }
  build_subtree_lists(S, rpt, sub_levels, P);
}

}  // namespace lobpcg

namespace lobpcg {

std::string verify_solve_plan(const Symbolic& S, const SolvePlan& P) {
  const int ns = S.nsuper;
  // the solve kernels use 64-row tiles and step the reduction 16 rows at a time from k0
  if (P.rows_per_tile != 64) return "solve plan tile rows";
  if ((int)P.fwd_wide.size() != S.nlevels || (int)P.bwd_wide.size() != S.nlevels) return "solve plan level modes";
  auto check_items = [&](const std::vector<int32_t>& items, const std::vector<int32_t>& fin, int64_t slots,
                         bool fwd) -> std::string {
    if (items.size() % kSolveItemInts != 0) return "solve item list size";
    for (size_t q = 0; q < items.size(); q += kSolveItemInts) {
      const int s = items[q], t = items[q + 1], k0 = items[q + 2], k1 = items[q + 3], slot = items[q + 4];
      if (s >= 0 && s < ns) {
        const int64_t po = (int64_t)(uint32_t)items[q + 8] | ((int64_t)items[q + 9] << 32);
        if (items[q + 5] != S.begin[s] || items[q + 6] != S.nr[s] || items[q + 7] != S.nc[s] ||
            po != S.panel_off[s] || items[q + 10] != (fwd ? S.uvec_off[s] : P.bwd_src_off[s]) ||
            items[q + 11] != (S.child_ptr[s + 1] > S.child_ptr[s] ? 1 : 0))
          return "solve item metadata";
      }
      if (s < 0 || s >= ns || t < 0) return "solve item supernode";
      const int lim = fwd ? S.nr[s] : S.nc[s];
      if (t * P.rows_per_tile >= lim) return "solve item tile";
      const int kl = fwd ? S.nc[s] : S.nr[s];
      if (k0 < 0 || k1 > kl || k0 >= k1 || k0 % 16 != 0) return "solve item K range";
      if (!fwd && k0 < t * P.rows_per_tile) return "backward K range below the diagonal tile";
      if (slot < -1 || slot >= slots) return "solve item slot";
    }
    for (size_t q = 0; q < fin.size(); q += 4) {
      const int s = fin[q], t = fin[q + 1], s0 = fin[q + 2], nch = fin[q + 3];
      if (s < 0 || s >= ns || t < 0 || s0 < 0 || nch < 2 || s0 + nch > slots) return "finalize item";
      if (t * P.rows_per_tile >= (fwd ? S.nr[s] : S.nc[s])) return "finalize tile";
    }
    return "";
  };
  if ((int)P.bwd_src_off.size() != ns) return "backward source list offsets";
  for (int s = 0; s < ns; ++s) {
    const int64_t o = P.bwd_src_off[s];
    if (o % 4 != 0 || o < 0 || o + panel_ld(S.nr[s]) > (int64_t)P.bwd_src.size()) return "backward source list range";
    for (int k = 0; k < S.nr[s]; ++k) {
      const int32_t v = P.bwd_src[o + k];
      if (v < 0 || v >= 2 * S.n || (k < S.nc[s]) != (v < S.n)) return "backward source row";
    }
  }
  if (P.gather_ptr.size() != P.gather_dst.size() + 1 || P.gather_ptr[0] != 0 ||
      (size_t)P.gather_ptr.back() != P.gather_src.size())
    return "gather list sizes";
  for (size_t i = 0; i < P.gather_dst.size(); ++i) {
    const int32_t d = P.gather_dst[i];
    if (d >= 0 ? d >= S.n : (int64_t)(-d - 1) >= S.uvec_total) return "gather destination";
    if (P.gather_ptr[i + 1] < P.gather_ptr[i]) return "gather pointers";
  }
  for (int32_t v : P.gather_src)
    if (v < 0 || v >= S.uvec_total) return "gather source";
  {
    std::string e = check_items(P.fwd_items, P.fwd_fin, P.fwd_slots, true);
    if (!e.empty()) return "forward " + e;
    e = check_items(P.bwd_items, P.bwd_fin, P.bwd_slots, false);
    if (!e.empty()) return "backward " + e;
  }
  // subtree lists
  if (P.sub_levels < 0 || P.sub_levels > S.nlevels) return "subtree levels";
  if (P.sub_levels > 0) {
    const int64_t ne = P.nsub * P.sub_levels + 1;
    if ((int64_t)P.sub_gather_off.size() != ne || (int64_t)P.sub_fwd_off.size() != ne ||
        (int64_t)P.sub_bwd_off.size() != ne)
      return "subtree offsets";
    for (int64_t e = 0; e + 1 < ne; ++e)
      if (P.sub_gather_off[e + 1] < P.sub_gather_off[e] || P.sub_fwd_off[e + 1] < P.sub_fwd_off[e] ||
          P.sub_bwd_off[e + 1] < P.sub_bwd_off[e])
        return "subtree offsets order";
    if (P.sub_gather_off[ne - 1] != (int64_t)P.sub_gather_dst.size() ||
        P.sub_fwd_off[ne - 1] * kSolveItemInts != (int64_t)P.sub_fwd_items.size() ||
        P.sub_bwd_off[ne - 1] * kSolveItemInts != (int64_t)P.sub_bwd_items.size())
      return "subtree list sizes";
    if (P.sub_gather_ptr.size() != P.sub_gather_dst.size() + 1 || P.sub_gather_ptr[0] != 0 ||
        (size_t)P.sub_gather_ptr.back() != P.sub_gather_src.size())
      return "subtree gather sizes";
    for (size_t i = 0; i < P.sub_gather_dst.size(); ++i) {
      const int32_t d = P.sub_gather_dst[i];
      if (d >= 0 ? d >= S.n : (int64_t)(-d - 1) >= S.uvec_total) return "subtree gather destination";
      if (P.sub_gather_ptr[i + 1] < P.sub_gather_ptr[i]) return "subtree gather pointers";
    }
    for (int32_t v : P.sub_gather_src)
      if (v < 0 || v >= S.uvec_total) return "subtree gather source";
    const std::vector<int32_t> nofin;
    std::string e = check_items(P.sub_fwd_items, nofin, 0, true);
    if (!e.empty()) return "subtree forward " + e;
    e = check_items(P.sub_bwd_items, nofin, 0, false);
    if (!e.empty()) return "subtree backward " + e;
    for (size_t q = 0; q < P.sub_fwd_items.size(); q += kSolveItemInts)
      if (S.level[P.sub_fwd_items[q]] >= P.sub_levels) return "subtree item level";
    for (size_t q = 0; q < P.sub_bwd_items.size(); q += kSolveItemInts)
      if (S.level[P.sub_bwd_items[q]] >= P.sub_levels) return "subtree item level";
  }
  return "";
}

std::string verify(const Symbolic& S, const FactorPlan& F, const SolvePlan& P, const std::vector<int32_t>& prow,
                   const std::vector<int32_t>& apos) {
  const int64_t n = S.n;
  const int ns = S.nsuper;
  auto ntiles = [](int64_t x) { return (int)((x + kTile - 1) / kTile); };
  if ((int64_t)S.perm.size() != n || (int64_t)S.iperm.size() != n) return "perm size";
  for (int64_t i = 0; i < n; ++i)
    if (S.perm[i] < 0 || S.perm[i] >= n || S.iperm[S.perm[i]] != i) return "perm/iperm mismatch";
  int64_t covered = 0;
  for (int s = 0; s < ns; ++s) {
    const int nc = S.nc[s], nr = S.nr[s], nb = nr - nc;
    if (nc < 1 || nb < 0) return "supernode size";
    if (S.begin[s] != covered) return "supernode columns not contiguous";
    covered += nc;
    if (S.row_off[s + 1] - S.row_off[s] != nr) return "row_off";
    const int32_t* r = &S.rows[S.row_off[s]];
    for (int t = 0; t < nc; ++t)
      if (r[t] != S.begin[s] + t) return "own rows";
    for (int j = nc; j < nr; ++j) {
      if (r[j] < S.begin[s] + nc || r[j] >= n) return "below row out of range";
      if (j > nc && r[j] <= r[j - 1]) return "below rows not increasing";
    }
    if (S.panel_off[s + 1] - S.panel_off[s] != panel_ld(nr) * nc) return "panel_off";
    if (S.upd_off[s + 1] - S.upd_off[s] != (int64_t)nb * nb) return "upd_off";
    if (S.uvec_off[s + 1] - S.uvec_off[s] != nb) return "uvec_off";
    if (S.dinv_off[s + 1] - S.dinv_off[s] != 2 * (int64_t)ntiles(nc) * kTile * kTile) return "dinv_off";
    if (S.lcopy_off[s] < 0 || S.lcopy_off[s] + 2 * (int64_t)nc * nc + (int64_t)(S.nr[s] - nc) * nc > S.lcopy_max)
      return "lcopy_off";
    const int p = S.parent[s];
    if (p >= 0) {
      if (p <= s || p >= ns) return "parent";
      if (S.level[p] <= S.level[s]) return "level order";
      if (S.inv_off[s + 1] - S.inv_off[s] != S.nr[p]) return "inv_off";
      for (int pos = 0; pos < S.nr[p]; ++pos) {
        const int32_t j = S.invmap[S.inv_off[s] + pos];
        if (j < -1 || j >= nb) return "invmap range";
        if (j >= 0 && S.relpos[S.row_off[s] + nc + j] != pos) return "invmap/relpos mismatch";
      }
      for (int j = 0; j < nb; ++j) {
        const int32_t pos = S.relpos[S.row_off[s] + nc + j];
        if (pos < 0 || pos >= S.nr[p]) return "relpos range";
        if (S.rows[S.row_off[p] + pos] != r[nc + j]) return "relpos target";
      }
    } else if (nb != 0) {
      return "root with below rows";
    }
  }
  if (covered != n) return "supernodes do not cover all columns";
  for (int s = 0; s < ns; ++s)
    for (int32_t q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q)
      if (S.child_list[q] < 0 || S.child_list[q] >= ns || S.parent[S.child_list[q]] != s) return "child list";
  // factor tasks
  for (const FactorPlan::Step& st : F.steps) {
    if (st.off < 0 || st.off + st.count > (int64_t)F.tasks.size() / 4) return "step range";
    if (st.level < 0 || st.level >= S.nlevels) return "step level";
    if (st.kind == kAssemble) continue;
    for (int64_t q = st.off; q < st.off + st.count; ++q) {
      const int s = F.tasks[4 * q], I = F.tasks[4 * q + 1], J = F.tasks[4 * q + 2], p = F.tasks[4 * q + 3];
      if (s < 0 || s >= ns || S.level[s] != st.level) return "task supernode";
      const int np = ntiles(S.nc[s]), rt = np + ntiles(S.nr[s] - S.nc[s]);
      if (st.kind == kInvPrep) {
        if (I < 0 || I >= S.nc[s]) return "invprep column";
        continue;
      }
      const bool plevel = (st.kind == kInvT1 || st.kind == kInvX21);   // p holds the recursion level
      if (p < 0 || (!plevel && p >= np) || I < 0 || I >= rt || J < 0 || J >= rt) return "task tile";
      if (st.kind == kSchur && !(J >= np && I >= J)) return "Schur tile order";
      if (st.kind == kSchur2 && !(J >= np && I >= J && (I - np) % 2 == 0 && (J - np) % 2 == 0 && rt - np >= F.schur_wide_tiles))
        return "Schur block order";
      if (st.kind == kUpdate && !((J > p + 1 && J < np && I >= J) || (I == p && J == p))) return "update tile order";
      if (st.kind == kUpdateRest) return "update step kind";
      if ((st.kind == kPotrf || st.kind == kTrsm || st.kind == kInvScale) && !(J == p && I >= p))
        return "trsm tile order";
      if (st.kind == kInvUpdate && !(J < p && I >= p)) return "inverse update tile order";
      if (st.kind == kInvT1 || st.kind == kInvX21) {
        if (p < 1 || p > 30 || I >= np || J >= np) return "inversion task";
        const int m = ((I >> p) << p) + (1 << (p - 1));
        if ((I >> p) != (J >> p) || !(J < m && m <= I)) return "inversion task blocks";
      }
      if (st.kind == kInvP21 && !(I >= np && J < np)) return "inverse product task";
    }
  }
  for (size_t q = 0; q < F.asm_items.size(); q += 2) {
    const int s = F.asm_items[q], t = F.asm_items[q + 1];
    if (s < 0 || s >= ns || t < 0 || t >= S.nr[s]) return "assembly item";
  }
  {
    const std::string e = verify_solve_plan(S, P);
    if (!e.empty()) return e;
  }
  if (!prow.empty()) {
    if ((int64_t)prow.size() != n + 1 || apos.size() != (size_t)prow[n]) return "assembly positions size";
    std::vector<int32_t> sn_of(n);
    for (int s = 0; s < ns; ++s)
      for (int t = 0; t < S.nc[s]; ++t) sn_of[S.begin[s] + t] = s;
    for (int64_t j = 0; j < n; ++j)
      for (int32_t e = prow[j]; e < prow[j + 1]; ++e)
        if (apos[e] < -1 || apos[e] >= S.nr[sn_of[j]]) return "assembly position";
  }
  return "";
}

}  // namespace lobpcg
