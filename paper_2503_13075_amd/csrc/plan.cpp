// Host planner (runs once per topology).
//
// Supplement section 3 of the ILVES paper: the constrained bonds form a graph
// G (atoms, constraints) that is usually disconnected; its line graph L(G)
// (one vertex per constraint, an edge when two constraints share an atom)
// has the sparsity pattern of the Newton matrix A (Eq. defA); a fill-reducing
// ordering is computed once and the factorisation is then reused every step.
//
// The GPU cost of a sparse LU on one workgroup is set by the chain of
// dependent load-and-update rounds through the elimination levels, so the
// planner compares a minimum-deficiency ordering (no fill on trees, but one
// level per bond along a chain) with a nested-dissection ordering (cut-vertex
// or BFS-level separators: logarithmic depth along chains, some fill) under a
// critical-path model and keeps the cheaper one.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>
#include <set>
#include <stdexcept>
#include <tuple>
#include <unordered_set>

namespace ilves {

std::string validate_topology(int32_t n_atoms, int32_t n_con, const int32_t* pairs, const double* d) {
  if (n_atoms <= 0) return "n_atoms must be positive";
  if (n_con < 0) return "n_constraints must be non-negative";
  if (n_con > 0 && (pairs == nullptr || d == nullptr)) return "pairs and d must not be NULL";
  std::unordered_set<uint64_t> seen;
  seen.reserve(static_cast<size_t>(n_con) * 2);
  for (int32_t k = 0; k < n_con; ++k) {
    int32_t a = pairs[2 * k], b = pairs[2 * k + 1];
    if (a < 0 || b < 0 || a >= n_atoms || b >= n_atoms)
      return "constraint " + std::to_string(k) + ": atom index out of range";
    if (a == b) return "constraint " + std::to_string(k) + ": both atoms are the same";
    if (!(d[k] > 0.0) || !std::isfinite(d[k]))
      return "constraint " + std::to_string(k) + ": distance must be positive and finite";
    uint64_t lo = static_cast<uint64_t>(std::min(a, b)), hi = static_cast<uint64_t>(std::max(a, b));
    if (!seen.insert((lo << 32) | hi).second)
      return "constraint " + std::to_string(k) + ": duplicate atom pair";
  }
  return std::string();
}

std::vector<std::vector<int32_t>> split_molecules(int32_t n_atoms, int32_t n_con, const int32_t* pairs,
                                                  std::vector<int32_t>& free_atoms) {
  std::vector<int32_t> parent(n_atoms);
  std::iota(parent.begin(), parent.end(), 0);
  std::function<int32_t(int32_t)> find = [&](int32_t x) {
    while (parent[x] != x) {
      parent[x] = parent[parent[x]];
      x = parent[x];
    }
    return x;
  };
  std::vector<char> used(n_atoms, 0);
  for (int32_t k = 0; k < n_con; ++k) {
    int32_t a = find(pairs[2 * k]), b = find(pairs[2 * k + 1]);
    used[pairs[2 * k]] = used[pairs[2 * k + 1]] = 1;
    if (a != b) parent[std::max(a, b)] = std::min(a, b);
  }
  std::vector<int32_t> mol_of_root(n_atoms, -1);
  std::vector<std::vector<int32_t>> mols;
  for (int32_t k = 0; k < n_con; ++k) {
    int32_t root = find(pairs[2 * k]);
    if (mol_of_root[root] < 0) {
      mol_of_root[root] = static_cast<int32_t>(mols.size());
      mols.emplace_back();
    }
    mols[mol_of_root[root]].push_back(k);
  }
  free_atoms.clear();
  for (int32_t i = 0; i < n_atoms; ++i)
    if (!used[i]) free_atoms.push_back(i);
  return mols;
}

// ---------------------------------------------------------------------------
// orderings

std::vector<int32_t> order_min_degree(const std::vector<std::vector<int32_t>>& adj) {
  // Minimum deficiency (fewest fill edges), ties broken by the elimination
  // level the vertex would get now (the deepest already-eliminated vertex it
  // depends on, plus one), then degree, then index.  On chordal graphs --
  // the line graph of a tree is one -- the simplicial vertices have
  // deficiency zero, so the order is a perfect elimination order and produces
  // no fill at all; the level tie-break peels all branches in step, which
  // keeps the elimination tree shallow (each level is a barrier on the GPU).
  const int32_t n = static_cast<int32_t>(adj.size());
  std::vector<std::vector<int32_t>> g = adj;
  auto has_edge = [&](int32_t a, int32_t b) { return std::binary_search(g[a].begin(), g[a].end(), b); };
  auto deficiency = [&](int32_t v) {
    int64_t miss = 0;
    const auto& nb = g[v];
    for (size_t i = 0; i < nb.size(); ++i)
      for (size_t j = i + 1; j < nb.size(); ++j)
        if (!has_edge(nb[i], nb[j])) ++miss;
    return miss;
  };
  using Key = std::tuple<int64_t, int32_t, int32_t, int32_t>;
  std::set<Key> pq;
  std::vector<Key> key(n);
  std::vector<int32_t> lev(n, 0);  // level v would get if eliminated now
  for (int32_t v = 0; v < n; ++v) {
    key[v] = Key{deficiency(v), 0, static_cast<int32_t>(g[v].size()), v};
    pq.insert(key[v]);
  }
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<int32_t> tmp, rest, touched;
  std::vector<char> mark(n, 0);
  while (!pq.empty()) {
    const int32_t v = std::get<3>(*pq.begin());
    pq.erase(pq.begin());
    order.push_back(v);
    const std::vector<int32_t> nb = g[v];
    for (int32_t u : nb) lev[u] = std::max(lev[u], lev[v] + 1);
    for (int32_t u : nb) {
      rest.clear();
      for (int32_t w : g[u])
        if (w != v) rest.push_back(w);
      tmp.clear();
      // g[u] <- (g[u] \ {v}) union (nb \ {u}); both sorted
      size_t i = 0, j = 0;
      while (i < rest.size() || j < nb.size()) {
        if (j < nb.size() && nb[j] == u) { ++j; continue; }
        if (j >= nb.size() || (i < rest.size() && rest[i] < nb[j])) tmp.push_back(rest[i++]);
        else if (i >= rest.size() || nb[j] < rest[i]) tmp.push_back(nb[j++]);
        else { tmp.push_back(rest[i]); ++i; ++j; }
      }
      g[u] = tmp;
    }
    g[v].clear();
    // deficiencies change within two hops of v
    touched.clear();
    for (int32_t u : nb) {
      if (!mark[u]) { mark[u] = 1; touched.push_back(u); }
      for (int32_t w : g[u])
        if (!mark[w]) { mark[w] = 1; touched.push_back(w); }
    }
    for (int32_t w : touched) {
      mark[w] = 0;
      pq.erase(key[w]);
      key[w] = Key{deficiency(w), lev[w], static_cast<int32_t>(g[w].size()), w};
      pq.insert(key[w]);
    }
  }
  return order;
}

namespace {

std::vector<int32_t> induced_md(const std::vector<std::vector<int32_t>>& adj, const std::vector<int32_t>& nodes,
                                std::vector<int32_t>& local_of) {
  for (size_t i = 0; i < nodes.size(); ++i) local_of[nodes[i]] = static_cast<int32_t>(i);
  std::vector<std::vector<int32_t>> sub(nodes.size());
  for (size_t i = 0; i < nodes.size(); ++i)
    for (int32_t u : adj[nodes[i]])
      if (local_of[u] >= 0) sub[i].push_back(local_of[u]);
  for (auto& s : sub) std::sort(s.begin(), s.end());
  std::vector<int32_t> o = order_min_degree(sub);
  for (int32_t v : nodes) local_of[v] = -1;
  std::vector<int32_t> out(o.size());
  for (size_t i = 0; i < o.size(); ++i) out[i] = nodes[o[i]];
  return out;
}

}  // namespace

std::vector<int32_t> order_nested_dissection(const std::vector<std::vector<int32_t>>& adj, int leaf) {
  const int32_t n = static_cast<int32_t>(adj.size());
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<int32_t> mark(n, -1), lev(n, -1), local_of(n, -1);
  // depth-first search state for the cut-vertex separators
  std::vector<int32_t> disc(n, -1), low(n, 0), sub(n, 0), par(n, -1), sepsum(n, 0), maxc(n, 0), nsep(n, 0);
  std::vector<std::pair<int32_t, int32_t>> stk;
  int32_t next_id = 0;
  std::vector<int32_t> queue;
  queue.reserve(n);

  // BFS restricted to vertices with mark == id; returns the visit order.
  auto bfs = [&](int32_t start, int32_t id) {
    queue.clear();
    queue.push_back(start);
    lev[start] = 0;
    for (size_t h = 0; h < queue.size(); ++h) {
      int32_t v = queue[h];
      for (int32_t u : adj[v])
        if (mark[u] == id && lev[u] < 0) {
          lev[u] = lev[v] + 1;
          queue.push_back(u);
        }
    }
    return queue;
  };

  std::function<void(const std::vector<int32_t>&)> rec = [&](const std::vector<int32_t>& nodes) {
    const int32_t sz = static_cast<int32_t>(nodes.size());
    if (sz <= leaf) {
      std::vector<int32_t> o = induced_md(adj, nodes, local_of);
      order.insert(order.end(), o.begin(), o.end());
      return;
    }
    const int32_t id = next_id++;
    for (int32_t v : nodes) mark[v] = id;
    std::vector<int32_t> sep;
    // 1) a single cut vertex that splits the part evenly: on the chains and
    //    trees of constraints a separator of one row, so the depth of the
    //    elimination tree grows with log(size) only
    {
      const int32_t root = nodes[0];
      for (int32_t v : nodes) {
        disc[v] = -1;
        sepsum[v] = 0;
        maxc[v] = 0;
        nsep[v] = 0;
      }
      int32_t timer = 0;
      disc[root] = low[root] = timer++;
      sub[root] = 1;
      par[root] = -1;
      stk.clear();
      stk.emplace_back(root, 0);
      while (!stk.empty()) {
        const int32_t v = stk.back().first;
        const int32_t it = stk.back().second;
        if (it < static_cast<int32_t>(adj[v].size())) {
          stk.back().second = it + 1;
          const int32_t u = adj[v][it];
          if (mark[u] != id) continue;
          if (disc[u] < 0) {
            par[u] = v;
            disc[u] = low[u] = timer++;
            sub[u] = 1;
            stk.emplace_back(u, 0);
          } else if (u != par[v]) {
            low[v] = std::min(low[v], disc[u]);
          }
        } else {
          stk.pop_back();
          const int32_t pv = par[v];
          if (pv >= 0) {
            low[pv] = std::min(low[pv], low[v]);
            sub[pv] += sub[v];
            if (low[v] >= disc[pv]) {  // v's subtree is cut off by removing pv
              sepsum[pv] += sub[v];
              maxc[pv] = std::max(maxc[pv], sub[v]);
              nsep[pv]++;
            }
          }
        }
      }
      int32_t best = -1, best_max = sz;
      if (timer == sz) {
        for (int32_t v : nodes) {
          const bool cut = v == root ? nsep[v] >= 2 : nsep[v] >= 1;
          if (!cut) continue;
          const int32_t mc = std::max(maxc[v], v == root ? 0 : sz - 1 - sepsum[v]);
          if (mc < best_max) {
            best_max = mc;
            best = v;
          }
        }
      }
      if (best >= 0 && 4 * best_max <= 3 * sz) sep.push_back(best);
    }
    if (sep.empty()) {
    // 2) otherwise a BFS level: pseudo-peripheral start vertex (George-Liu style)
    int32_t start = nodes[0];
    int32_t ecc = -1;
    for (int rep = 0; rep < 4; ++rep) {
      for (int32_t v : nodes) lev[v] = -1;
      std::vector<int32_t> vis = bfs(start, id);
      int32_t e = lev[vis.back()];
      if (e <= ecc) break;
      ecc = e;
      int32_t best = vis.back();
      for (int32_t v : vis)
        if (lev[v] == e && adj[v].size() < adj[best].size()) best = v;
      start = best;
    }
    for (int32_t v : nodes) lev[v] = -1;
    std::vector<int32_t> vis = bfs(start, id);
    const int32_t d = lev[vis.back()];
    if (d < 2 || static_cast<int32_t>(vis.size()) != sz) {
      for (int32_t v : nodes) {
        mark[v] = -1;
        lev[v] = -1;
      }
      std::vector<int32_t> o = induced_md(adj, nodes, local_of);
      order.insert(order.end(), o.begin(), o.end());
      return;
    }
    std::vector<int32_t> cnt(d + 1, 0);
    for (int32_t v : nodes) cnt[lev[v]]++;
    std::vector<int32_t> below(d + 2, 0);
    for (int32_t l = 0; l <= d; ++l) below[l + 1] = below[l] + cnt[l];
    int32_t best_l = -1;
    double best_score = 1e300;
    for (int32_t l = 1; l < d; ++l) {
      int32_t lo = below[l], hi = sz - below[l + 1];
      double bal = static_cast<double>(std::min(lo, hi)) / sz;
      if (bal < 0.2) continue;
      double score = cnt[l] * (1.0 + 2.0 * (0.5 - bal));
      if (score < best_score) { best_score = score; best_l = l; }
    }
    if (best_l < 0) best_l = d / 2;
    // separator: level best_l vertices that touch level best_l + 1
    for (int32_t v : nodes)
      if (lev[v] == best_l) {
        bool touches = false;
        for (int32_t u : adj[v])
          if (mark[u] == id && lev[u] == best_l + 1) { touches = true; break; }
        if (touches) sep.push_back(v);
      }
    }
    for (int32_t v : sep) mark[v] = -2;  // excluded from the parts
    // connected components of the rest
    std::vector<std::vector<int32_t>> parts;
    for (int32_t v : nodes) lev[v] = -1;
    for (int32_t v : nodes) {
      if (mark[v] != id || lev[v] >= 0) continue;
      std::vector<int32_t> comp = bfs(v, id);
      parts.push_back(comp);
    }
    for (int32_t v : nodes) {
      lev[v] = -1;
      if (mark[v] == id) mark[v] = -1;
    }
    for (auto& p : parts) rec(p);
    for (int32_t v : sep) mark[v] = -1;
    std::vector<int32_t> o = induced_md(adj, sep, local_of);
    order.insert(order.end(), o.begin(), o.end());
  };

  // each connected component separately
  std::vector<char> seen(n, 0);
  for (int32_t v = 0; v < n; ++v) {
    if (seen[v]) continue;
    std::vector<int32_t> comp{v};
    seen[v] = 1;
    for (size_t h = 0; h < comp.size(); ++h)
      for (int32_t u : adj[comp[h]])
        if (!seen[u]) {
          seen[u] = 1;
          comp.push_back(u);
        }
    rec(comp);
  }
  return order;
}

// ---------------------------------------------------------------------------
// symbolic factorisation

namespace {

struct Symbolic {
  std::vector<std::vector<int32_t>> up, low;  // strict upper / lower structure per row
  std::vector<int32_t> level;
  int32_t n_levels = 0;
  int32_t h_int = 0;  // levels holding the rows before the tail
  int64_t nnz_off = 0;
  double cost = 0.0;
};

// adj: adjacency in the permuted numbering.  The last n_tail rows (border
// rows of a part) are held back to levels after every other row.
Symbolic symbolic(const std::vector<std::vector<int32_t>>& adj, int32_t n_tail = 0) {
  const int32_t n = static_cast<int32_t>(adj.size());
  Symbolic S;
  S.up.resize(n);
  S.low.resize(n);
  S.level.assign(n, 0);
  for (int32_t p = 0; p < n; ++p)
    for (int32_t q : adj[p])
      if (q > p) S.up[p].push_back(q);
  for (int32_t p = 0; p < n; ++p) {
    auto& u = S.up[p];
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    if (!u.empty()) {
      auto& par = S.up[u[0]];  // elimination-tree parent inherits the rest
      par.insert(par.end(), u.begin() + 1, u.end());
    }
  }
  const int32_t n_int = n - n_tail;
  S.h_int = 0;
  for (int32_t p = 0; p < n; ++p) {
    if (p < n_int) S.h_int = std::max(S.h_int, S.level[p] + 1);
    else S.level[p] = std::max(S.level[p], S.h_int);  // every interior level is final here
    for (int32_t q : S.up[p]) {
      S.low[q].push_back(p);
      S.level[q] = std::max(S.level[q], S.level[p] + 1);
    }
  }
  for (int32_t p = 0; p < n; ++p) {
    S.n_levels = std::max(S.n_levels, S.level[p] + 1);
    S.nnz_off += static_cast<int64_t>(S.up[p].size());
  }
  // Cost model (critical path of the level-scheduled sweeps, fitted to
  // measured solve times): a level costs a fixed part LEVEL (barrier and
  // bookkeeping) plus the longest chain of dependent load-and-update rounds
  // of any of its items -- a row takes one round per BATCH lower entries, a
  // pair task one per update, and a wave that holds both kinds runs them one
  // after the other; levels wider than LANES take several passes.  The
  // backward sweep walks the levels again with one round per BATCH upper
  // entries.
  const double LEVEL = 0.7, BATCH = 2.0, LANES = 256.0;
  std::vector<int32_t> max_row(S.n_levels, 0), max_pair(S.n_levels, 0), max_back(S.n_levels, 0);
  std::vector<int64_t> items(S.n_levels, 0);
  std::vector<int32_t> in_low(n, -1);
  for (int32_t j = 0; j < n; ++j) {
    const int32_t h = S.level[j];
    if (h > 0) {
      max_row[h] = std::max(max_row[h], static_cast<int32_t>(std::ceil(S.low[j].size() / BATCH)));
      for (int32_t i : S.low[j]) in_low[i] = j;
      for (int32_t m : S.up[j]) {
        int32_t common = 0;
        for (int32_t i : S.low[m])
          if (in_low[i] == j) ++common;
        if (common > 0) {
          max_pair[h] = std::max(max_pair[h], common);
          ++items[h];
        }
      }
      ++items[h];
    }
    max_back[h] = std::max(max_back[h], static_cast<int32_t>(std::ceil(S.up[j].size() / BATCH)));
  }
  for (int32_t h = 0; h < S.n_levels; ++h) {
    const double passes = std::max(1.0, std::ceil(static_cast<double>(items[h]) / LANES));
    if (h > 0) S.cost += LEVEL + passes * (max_row[h] + max_pair[h]);
    S.cost += LEVEL + max_back[h];
  }
  return S;
}

std::vector<std::vector<int32_t>> permute_graph(const std::vector<std::vector<int32_t>>& adj,
                                                const std::vector<int32_t>& perm) {
  const int32_t n = static_cast<int32_t>(adj.size());
  std::vector<int32_t> inv(n);
  for (int32_t p = 0; p < n; ++p) inv[perm[p]] = p;
  std::vector<std::vector<int32_t>> out(n);
  for (int32_t p = 0; p < n; ++p) {
    for (int32_t u : adj[perm[p]]) out[p].push_back(inv[u]);
    std::sort(out[p].begin(), out[p].end());
  }
  return out;
}

int32_t find_sorted(const std::vector<int32_t>& v, int32_t x) {
  auto it = std::lower_bound(v.begin(), v.end(), x);
  return static_cast<int32_t>(it - v.begin());
}

}  // namespace

MolPlan plan_molecule(const std::vector<int32_t>& cons, const int32_t* pairs, const double* d,
                      const PlanOptions& opt, const PartSpec* part) {
  MolPlan P;
  const int32_t n = static_cast<int32_t>(cons.size());
  const int32_t n_tail = part ? part->n_tail : 0;
  const int32_t n_int = n - n_tail;
  P.n = n;
  // local atoms (a part's own atoms first, each run sorted)
  std::vector<int32_t> atoms;
  atoms.reserve(2 * n);
  for (int32_t c : cons) {
    atoms.push_back(pairs[2 * c]);
    atoms.push_back(pairs[2 * c + 1]);
  }
  std::sort(atoms.begin(), atoms.end());
  atoms.erase(std::unique(atoms.begin(), atoms.end()), atoms.end());
  int32_t s_own = static_cast<int32_t>(atoms.size());
  if (part && part->owned) {
    const std::vector<int32_t>& own = *part->owned;
    std::vector<int32_t> rest;
    for (int32_t a : atoms)
      if (!std::binary_search(own.begin(), own.end(), a)) rest.push_back(a);
    s_own = static_cast<int32_t>(own.size());
    atoms = own;
    atoms.insert(atoms.end(), rest.begin(), rest.end());
  }
  P.s = static_cast<int32_t>(atoms.size());
  P.s_own = s_own;
  P.atom_gid = atoms;
  auto local_atom = [&](int32_t g) {
    auto it = std::lower_bound(atoms.begin(), atoms.begin() + s_own, g);
    if (it != atoms.begin() + s_own && *it == g) return static_cast<int32_t>(it - atoms.begin());
    return static_cast<int32_t>(std::lower_bound(atoms.begin() + s_own, atoms.end(), g) - atoms.begin());
  };
  std::vector<int32_t> la(n), lb(n);
  for (int32_t c = 0; c < n; ++c) {
    la[c] = local_atom(pairs[2 * cons[c]]);
    lb[c] = local_atom(pairs[2 * cons[c] + 1]);
  }
  // incidence (local constraint order) and line graph
  std::vector<std::vector<int32_t>> inc(P.s);
  for (int32_t c = 0; c < n; ++c) {
    inc[la[c]].push_back(c);
    inc[lb[c]].push_back(c);
  }
  std::vector<std::vector<int32_t>> adj(n);
  for (int32_t x = 0; x < P.s; ++x)
    for (size_t i = 0; i < inc[x].size(); ++i)
      for (size_t j = 0; j < inc[x].size(); ++j)
        if (i != j) adj[inc[x][i]].push_back(inc[x][j]);
  int64_t n_edges = 0;
  for (auto& a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
    n_edges += static_cast<int64_t>(a.size());
  }
  n_edges /= 2;

  // ordering (of a part: its interior rows, the border rows after them)
  std::vector<std::vector<int32_t>> adj_int;
  if (n_tail > 0) {
    adj_int.resize(n_int);
    for (int32_t c = 0; c < n_int; ++c)
      for (int32_t x : adj[c])
        if (x < n_int) adj_int[c].push_back(x);
  }
  const std::vector<std::vector<int32_t>>& adj_o = n_tail > 0 ? adj_int : adj;
  auto with_tail = [&](std::vector<int32_t> pm) {
    for (int32_t c = n_int; c < n; ++c) pm.push_back(c);
    return pm;
  };
  std::vector<int32_t> perm = with_tail(order_min_degree(adj_o));
  Symbolic S = symbolic(permute_graph(adj, perm), n_tail);
  P.ordering = 1;
  if (opt.ordering == 2 || (opt.ordering == 0 && n_int > 2 * opt.nd_leaf)) {
    std::vector<int32_t> perm_nd = with_tail(order_nested_dissection(adj_o, opt.nd_leaf));
    Symbolic Snd = symbolic(permute_graph(adj, perm_nd), n_tail);
    if (opt.ordering == 2 || Snd.cost < S.cost) {
      perm = perm_nd;
      S = std::move(Snd);
      P.ordering = 2;
    }
  }
  // Renumber rows by elimination level (stable within a level).  Any
  // topological order of the elimination tree is an equivalent ordering:
  // same filled pattern, same tree, same levels.
  {
    std::vector<int32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return S.level[a] < S.level[b]; });
    std::vector<int32_t> perm2(n);
    for (int32_t p = 0; p < n; ++p) perm2[p] = perm[idx[p]];
    const int64_t nnz_before = S.nnz_off;
    const int32_t lev_before = S.n_levels;
    perm = perm2;
    S = symbolic(permute_graph(adj, perm), n_tail);
    if (S.nnz_off != nnz_before || S.n_levels != lev_before)
      throw std::logic_error("level renumbering changed the filled pattern");
    for (int32_t p = 1; p < n; ++p)
      if (S.level[p] < S.level[p - 1]) throw std::logic_error("rows are not sorted by level");
    for (int32_t p = n_int; p < n; ++p)
      if (perm[p] < n_int) throw std::logic_error("a border row moved before an interior row");
  }
  std::vector<int32_t> inv(n);
  for (int32_t p = 0; p < n; ++p) inv[perm[p]] = p;
  P.n_levels = S.n_levels;
  P.n_int = n_int;
  P.h_int = n_tail > 0 ? S.h_int : S.n_levels;
  P.fill = S.nnz_off - n_edges;
  P.cost = S.cost;

  P.cid.resize(n);
  P.ra.resize(n);
  P.rb.resize(n);
  P.d2.resize(n);
  for (int32_t p = 0; p < n; ++p) {
    const int32_t c = perm[p];
    P.cid[p] = cons[c];
    P.ra[p] = la[c];
    P.rb[p] = lb[c];
    P.d2[p] = d[cons[c]] * d[cons[c]];
  }
  // slot regions
  P.up_start.assign(n + 1, 0);
  P.l_start.assign(n + 1, 0);
  for (int32_t p = 0; p < n; ++p) P.up_start[p + 1] = P.up_start[p] + static_cast<int32_t>(S.up[p].size());
  P.n_up = P.up_start[n];
  P.l_start[0] = P.n_up;
  for (int32_t p = 0; p < n; ++p) P.l_start[p + 1] = P.l_start[p] + static_cast<int32_t>(S.low[p].size());
  P.n_l = P.l_start[n] - P.n_up;
  auto up_slot = [&](int32_t j, int32_t m) { return P.up_start[j] + find_sorted(S.up[j], m); };   // m > j
  auto l_slot = [&](int32_t k, int32_t i) { return P.l_start[k] + find_sorted(S.low[k], i); };   // i < k
  auto coupling = [&](int32_t k, int32_t j) -> int32_t {
    const int32_t ck = perm[k], cj = perm[j];
    int32_t x = -1;
    if (la[ck] == la[cj] || la[ck] == lb[cj]) x = la[ck];
    else if (lb[ck] == la[cj] || lb[ck] == lb[cj]) x = lb[ck];
    if (x < 0) return P.s << 1;  // fill: zero coupling (sentinel atom)
    const int sk = (x == la[ck]) ? 1 : -1;
    const int sj = (x == la[cj]) ? 1 : -1;
    return (x << 1) | ((sk * sj) < 0 ? 1 : 0);
  };
  P.ucol.assign(P.n_up, 0);
  P.utr.assign(P.n_up, 0);
  P.ucoef.assign(P.n_up, 0);
  P.ustart.assign(P.n_up + 1, 0);
  P.lcol.assign(P.n_l, 0);
  P.ltr.assign(P.n_l, 0);
  P.lcoef.assign(P.n_l, 0);
  for (int32_t j = 0; j < n; ++j) {
    for (size_t t = 0; t < S.up[j].size(); ++t) {
      const int32_t m = S.up[j][t];
      const int32_t q = P.up_start[j] + static_cast<int32_t>(t);
      P.ucol[q] = m;
      P.utr[q] = l_slot(m, j);
      P.ucoef[q] = coupling(j, m);
      // rows i < j coupled to both j and m: low(j) intersect low(m)
      const auto& A = S.low[j];
      const auto& B = S.low[m];
      size_t ia = 0, ib = 0;
      while (ia < A.size() && ib < B.size()) {
        if (A[ia] < B[ib]) ++ia;
        else if (B[ib] < A[ia]) ++ib;
        else {
          P.upd_a.push_back(l_slot(j, A[ia]));
          P.upd_b.push_back(l_slot(m, B[ib]));
          ++ia;
          ++ib;
        }
      }
      P.ustart[q + 1] = static_cast<int32_t>(P.upd_a.size());
    }
    for (size_t t = 0; t < S.low[j].size(); ++t) {
      const int32_t i = S.low[j][t];
      const int32_t q = P.l_start[j] + static_cast<int32_t>(t) - P.n_up;
      P.lcol[q] = i;
      P.ltr[q] = up_slot(i, j);
      P.lcoef[q] = coupling(j, i);
    }
  }
  P.n_upd = static_cast<int32_t>(P.upd_a.size());
  P.lvl_row.assign(S.n_levels + 1, n);
  P.lvl_row[0] = 0;
  for (int32_t p = n - 1; p >= 0; --p) P.lvl_row[S.level[p]] = p;
  P.pl_start.assign(S.n_levels + 1, 0);
  for (int32_t h = 0; h < S.n_levels; ++h) {
    for (int32_t q = P.up_start[P.lvl_row[h]]; q < P.up_start[P.lvl_row[h + 1]]; ++q)
      if (P.ustart[q + 1] > P.ustart[q]) P.plist.push_back(q);
    P.pl_start[h + 1] = static_cast<int32_t>(P.plist.size());
  }
  for (int32_t p = 0; p < n; ++p) {
    if (S.level[p] == 0 && !S.low[p].empty()) throw std::logic_error("level-0 rows must have no lower entries");
    if (p < n_int && S.level[p] > 0 && S.low[p].empty()) throw std::logic_error("rows without lower entries must be at level 0");
    if ((p < n_int) != (S.level[p] < P.h_int)) throw std::logic_error("border rows must sit alone in the last levels");
  }
  // incidence in elimination order
  P.inc_ptr.assign(P.s + 1, 0);
  for (int32_t x = 0; x < P.s; ++x) P.inc_ptr[x + 1] = P.inc_ptr[x] + static_cast<int32_t>(inc[x].size());
  P.inc.resize(P.inc_ptr[P.s]);
  for (int32_t x = 0; x < P.s; ++x) {
    std::vector<int32_t> rows;
    for (int32_t c : inc[x]) rows.push_back(inv[c]);
    std::sort(rows.begin(), rows.end());
    for (size_t t = 0; t < rows.size(); ++t) {
      const int32_t p = rows[t];
      P.inc[P.inc_ptr[x] + t] = (p << 1) | (P.rb[p] == x ? 1 : 0);
    }
  }
  return P;
}

// ---------------------------------------------------------------------------
// split of one molecule across several workgroups

namespace {

// Groups of atoms of about `target` constraints each, from a breadth-first
// spanning tree of the bond graph rooted at a peripheral atom: walking the
// tree bottom-up, a subtree is cut off as a group once it holds `target`
// constraints (each constraint counts at its endpoint found later by the
// search), and a vertex whose uncut children together exceed 1.5 target
// first cuts its heaviest children.  Groups are numbered in search order of
// their roots, so neighbouring groups of a chain get consecutive numbers.
std::vector<int32_t> group_atoms(int32_t s, const std::vector<int32_t>& la, const std::vector<int32_t>& lb,
                                 int32_t target, int32_t& n_groups) {
  const int32_t n = static_cast<int32_t>(la.size());
  std::vector<std::vector<int32_t>> nb(s);
  for (int32_t c = 0; c < n; ++c) {
    nb[la[c]].push_back(lb[c]);
    nb[lb[c]].push_back(la[c]);
  }
  auto bfs = [&](int32_t root, std::vector<int32_t>& order, std::vector<int32_t>& parent) {
    order.assign(1, root);
    parent.assign(s, -2);
    parent[root] = -1;
    for (size_t h = 0; h < order.size(); ++h)
      for (int32_t y : nb[order[h]])
        if (parent[y] == -2) {
          parent[y] = order[h];
          order.push_back(y);
        }
  };
  std::vector<int32_t> order, parent;
  bfs(0, order, parent);
  bfs(order.back(), order, parent);  // from an atom at the far end
  std::vector<int32_t> pos(s);
  for (int32_t h = 0; h < s; ++h) pos[order[h]] = h;
  std::vector<double> resid(s, 0.0), added(s, 0.0);
  for (int32_t c = 0; c < n; ++c) resid[pos[la[c]] > pos[lb[c]] ? la[c] : lb[c]] += 1.0;
  std::vector<std::vector<int32_t>> kids(s);
  for (int32_t v : order)
    if (parent[v] >= 0) kids[parent[v]].push_back(v);
  std::vector<char> cut(s, 0);
  const double T = static_cast<double>(target);
  for (int32_t h = s - 1; h >= 0; --h) {
    const int32_t v = order[h];
    while (resid[v] > 1.5 * T) {
      int32_t best = -1;
      for (int32_t k : kids[v])
        if (!cut[k] && added[k] > 0.0 && (best < 0 || added[k] > added[best])) best = k;
      if (best < 0) break;
      cut[best] = 1;
      resid[v] -= added[best];
    }
    if (parent[v] >= 0 && resid[v] >= T) {
      cut[v] = 1;
    } else if (parent[v] >= 0) {
      added[v] = resid[v];
      resid[parent[v]] += resid[v];
    }
  }
  std::vector<int32_t> group(s, -1);
  n_groups = 0;
  for (int32_t v : order) group[v] = (parent[v] < 0 || cut[v]) ? n_groups++ : group[parent[v]];
  return group;
}

}  // namespace

bool plan_split(const std::vector<int32_t>& cons, const int32_t* pairs, const double* d, const PlanOptions& opt,
                int32_t part_rows, SplitPlan& out) {
  const int32_t n = static_cast<int32_t>(cons.size());
  std::vector<int32_t> atoms;
  for (int32_t c : cons) {
    atoms.push_back(pairs[2 * c]);
    atoms.push_back(pairs[2 * c + 1]);
  }
  std::sort(atoms.begin(), atoms.end());
  atoms.erase(std::unique(atoms.begin(), atoms.end()), atoms.end());
  const int32_t s = static_cast<int32_t>(atoms.size());
  std::vector<int32_t> la(n), lb(n);
  for (int32_t c = 0; c < n; ++c) {
    la[c] = find_sorted(atoms, pairs[2 * cons[c]]);
    lb[c] = find_sorted(atoms, pairs[2 * cons[c] + 1]);
  }
  int32_t G = 0;
  std::vector<int32_t> group = group_atoms(s, la, lb, std::max<int32_t>(part_rows, 8), G);
  // a group without interior constraints joins the group across its first
  // separator constraint (repeated until every group has some)
  for (int round = 0; round < G; ++round) {
    std::vector<int32_t> inner(G, 0);
    for (int32_t c = 0; c < n; ++c)
      if (group[la[c]] == group[lb[c]]) ++inner[group[la[c]]];
    int32_t bad = -1;
    for (int32_t g = 0; g < G && bad < 0; ++g)
      if (inner[g] == 0) bad = g;
    if (bad < 0) break;
    int32_t into = -1;
    for (int32_t c = 0; c < n && into < 0; ++c) {
      if (group[la[c]] == bad && group[lb[c]] != bad) into = group[lb[c]];
      else if (group[lb[c]] == bad && group[la[c]] != bad) into = group[la[c]];
    }
    if (into < 0) break;
    std::vector<int32_t> relabel(G);
    int32_t k = 0;
    for (int32_t g = 0; g < G; ++g) relabel[g] = g == bad ? -1 : k++;
    for (int32_t& g : group) g = g == bad ? relabel[into] : relabel[g];
    G = k;
  }
  if (G < 2 || G > kSplitMaxParts) return false;
  std::vector<std::vector<int32_t>> interior(G), border(G), owned(G);
  std::vector<int32_t> sep;  // local constraint indices of the separator rows
  for (int32_t c = 0; c < n; ++c) {
    const int32_t ga = group[la[c]], gb = group[lb[c]];
    if (ga == gb) {
      interior[ga].push_back(c);
    } else {
      sep.push_back(c);
      border[ga].push_back(c);
      border[gb].push_back(c);
    }
  }
  const int32_t m = static_cast<int32_t>(sep.size());
  if (m > kSplitMaxSep) return false;
  // separator rows ordered by their pair of parts: with groups numbered
  // along the molecule the separator matrix is then banded
  std::stable_sort(sep.begin(), sep.end(), [&](int32_t x, int32_t y) {
    const int32_t x0 = std::min(group[la[x]], group[lb[x]]), x1 = std::max(group[la[x]], group[lb[x]]);
    const int32_t y0 = std::min(group[la[y]], group[lb[y]]), y1 = std::max(group[la[y]], group[lb[y]]);
    return x0 != y0 ? x0 < y0 : x1 < y1;
  });
  for (int32_t g = 0; g < G; ++g)
    if (interior[g].empty() || static_cast<int32_t>(border[g].size()) > kSplitMaxBorder) return false;
  for (int32_t x = 0; x < s; ++x) owned[group[x]].push_back(atoms[x]);  // sorted, as atoms is

  SplitPlan S;
  S.m = m;
  S.parts.resize(G);
  std::vector<std::vector<int32_t>> row_of(G);  // per part: local constraint -> local row (or -1)
  // Parts take nested dissection unless an ordering is forced: every part of
  // a molecule waits at the barriers for the one with the most levels, and
  // the parts whose factor does not fit in LDS read their structure from
  // global memory level by level, where the level count dominates more than
  // the cost model (fitted to molecules held in LDS) assumes.
  PlanOptions part_opt = opt;
  if (part_opt.ordering == 0) part_opt.ordering = 2;
  for (int32_t g = 0; g < G; ++g) {
    std::vector<int32_t> pc;
    for (int32_t c : interior[g]) pc.push_back(cons[c]);
    for (int32_t c : border[g]) pc.push_back(cons[c]);
    PartSpec spec;
    spec.n_tail = static_cast<int32_t>(border[g].size());
    spec.owned = &owned[g];
    S.parts[g] = plan_molecule(pc, pairs, d, part_opt, &spec);
    const MolPlan& M = S.parts[g];
    if (M.n_int != static_cast<int32_t>(interior[g].size())) throw std::logic_error("part row count");
    row_of[g].assign(n, -1);
    for (int32_t p = 0; p < M.n; ++p) {
      const int32_t c = static_cast<int32_t>(std::lower_bound(cons.begin(), cons.end(), M.cid[p]) - cons.begin());
      row_of[g][c] = p;
    }
  }
  std::vector<int32_t> sep_index(n, -1);
  for (int32_t b = 0; b < m; ++b) sep_index[sep[b]] = b;
  S.sep_cid.resize(m);
  S.sep_ga.resize(m);
  S.sep_gb.resize(m);
  S.sep_part.resize(2 * m);
  S.sep_loc.resize(2 * m);
  for (int32_t b = 0; b < m; ++b) {
    const int32_t c = sep[b];
    S.sep_cid[b] = cons[c];
    S.sep_ga[b] = atoms[la[c]];
    S.sep_gb[b] = atoms[lb[c]];
    const int32_t g0 = std::min(group[la[c]], group[lb[c]]), g1 = std::max(group[la[c]], group[lb[c]]);
    S.sep_part[2 * b] = g0;
    S.sep_part[2 * b + 1] = g1;
    S.sep_loc[2 * b] = row_of[g0][c] - S.parts[g0].n_int;
    S.sep_loc[2 * b + 1] = row_of[g1][c] - S.parts[g1].n_int;
  }
  // constraint incidence of the atoms, for couplings
  std::vector<std::vector<int32_t>> inc(s);
  for (int32_t c = 0; c < n; ++c) {
    inc[la[c]].push_back(c);
    inc[lb[c]].push_back(c);
  }
  auto coupling = [&](int32_t x, int32_t c1, int32_t c2) {
    const int s1 = la[c1] == x ? 1 : -1, s2 = la[c2] == x ? 1 : -1;
    return (atoms[x] << 1) | (s1 * s2 < 0 ? 1 : 0);
  };
  S.sadj_ptr.assign(1, 0);
  for (int32_t b = 0; b < m; ++b) {
    const int32_t c = sep[b];
    for (int32_t x : {la[c], lb[c]})
      for (int32_t c2 : inc[x])
        if (c2 != c && sep_index[c2] >= 0) {
          S.sadj_col.push_back(sep_index[c2]);
          S.sadj_coef.push_back(coupling(x, c, c2));
        }
    S.sadj_ptr.push_back(static_cast<int32_t>(S.sadj_col.size()));
  }
  // half-bandwidth of the separator matrix after elimination without
  // pivoting: entries between rows that share an atom or a part, plus fill
  {
    std::vector<std::vector<char>> nz(m, std::vector<char>(m, 0));
    for (int32_t b = 0; b < m; ++b) {
      nz[b][b] = 1;
      for (int32_t a = S.sadj_ptr[b]; a < S.sadj_ptr[b + 1]; ++a) nz[b][S.sadj_col[a]] = 1;
      for (int32_t c = 0; c < m; ++c)
        for (int u = 0; u < 2; ++u)
          for (int v = 0; v < 2; ++v)
            if (S.sep_part[2 * b + u] == S.sep_part[2 * c + v]) nz[b][c] = 1;
    }
    for (int32_t p = 0; p < m; ++p)
      for (int32_t q = p + 1; q < m; ++q)
        if (nz[q][p])
          for (int32_t c = p + 1; c < m; ++c)
            if (nz[p][c]) nz[q][c] = 1;
    S.bw = 0;
    for (int32_t b = 0; b < m; ++b)
      for (int32_t c = 0; c < m; ++c)
        if (nz[b][c]) S.bw = std::max(S.bw, std::abs(b - c));
  }
  // rows coupled to a border row that its part does not hold
  S.ext_ptr.resize(G);
  S.ext_part.resize(G);
  S.ext_row.resize(G);
  S.ext_coef.resize(G);
  for (int32_t g = 0; g < G; ++g) {
    const MolPlan& M = S.parts[g];
    S.ext_ptr[g].assign(1, 0);
    for (int32_t p = M.n_int; p < M.n; ++p) {
      const int32_t c = static_cast<int32_t>(std::lower_bound(cons.begin(), cons.end(), M.cid[p]) - cons.begin());
      for (int32_t x : {la[c], lb[c]})
        for (int32_t c2 : inc[x]) {
          if (c2 == c || row_of[g][c2] >= 0) continue;
          // held by the part of its interior group, or (separator row) by its owner
          const int32_t h = sep_index[c2] >= 0 ? S.sep_part[2 * sep_index[c2]] : group[la[c2]];
          if (row_of[h][c2] < 0) throw std::logic_error("coupled row not held by its part");
          S.ext_part[g].push_back(h);
          S.ext_row[g].push_back(row_of[h][c2]);
          S.ext_coef[g].push_back(coupling(x, c, c2));
        }
      S.ext_ptr[g].push_back(static_cast<int32_t>(S.ext_part[g].size()));
    }
  }
  out = std::move(S);
  return true;
}

bool plan_split_auto(const std::vector<int32_t>& cons, const int32_t* pairs, const double* d,
                     const PlanOptions& opt, int32_t part_rows, SplitPlan& out) {
  if (part_rows > 0) return plan_split(cons, pairs, d, opt, part_rows, out);
  const int32_t n = static_cast<int32_t>(cons.size());
  for (int32_t rows = std::min(1024, std::max(384, n / 12)); rows <= 4096; rows = rows * 3 / 2)
    if (plan_split(cons, pairs, d, opt, rows, out)) return true;
  return false;
}

}  // namespace ilves
