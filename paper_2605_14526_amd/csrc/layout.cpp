// Host-side vertex ordering for the partitioned inverse: nested dissection by
// coordinate bisection with vertex separators.  The free vertices are split
// recursively at the median coordinate of the longest bounding-box axis; the
// vertices of the lower half that touch the upper half form the separator.
// Recursion stops at subdomains of at most max_sub vertices.  No subdomain
// vertex is adjacent to another subdomain, so A~ restricted to the subdomains
// is block diagonal and its Schur complement lives on the separators only.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

#include "pd_internal.h"

namespace pdhot {

namespace {

struct Graph {
  std::vector<int> ptr, adj;  // over all vertices, free-free edges only
};

Graph free_graph(int nv, int ne, const int32_t* tets, const uint8_t* pinned) {
  std::vector<std::vector<int>> nb(nv);
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int u = tets[4 * e + a], v = tets[4 * e + b];
        if (u != v && !pinned[u] && !pinned[v]) nb[u].push_back(v);
      }
  Graph g;
  g.ptr.assign(nv + 1, 0);
  for (int v = 0; v < nv; ++v) {
    auto& l = nb[v];
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
    g.ptr[v + 1] = g.ptr[v] + (int)l.size();
  }
  g.adj.reserve(g.ptr[nv]);
  for (int v = 0; v < nv; ++v) g.adj.insert(g.adj.end(), nb[v].begin(), nb[v].end());
  return g;
}

struct ND {
  const double* X;
  const Graph* g;
  int max_sub;
  std::vector<int> side;  // scratch membership marks
  std::vector<std::vector<int>> subs;
  // separator nodes in post-order (children before their parent) and the
  // separator nodes directly below each one
  std::vector<std::vector<int>> seps, kids;

  // Dissects `set`; returns the separator nodes at the top of its subtree
  // (none for a subdomain, two or more where a split found no separator).
  std::vector<int> run(std::vector<int> set) {
    if ((int)set.size() <= max_sub) {
      if (!set.empty()) subs.push_back(std::move(set));
      return {};
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v : set)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], X[3 * v + a]);
        hi[a] = std::max(hi[a], X[3 * v + a]);
      }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    std::vector<int> sorted = set;
    std::stable_sort(sorted.begin(), sorted.end(), [&](int a, int b) { return X[3 * a + ax] < X[3 * b + ax]; });
    double cval = X[3 * sorted[sorted.size() / 2] + ax];
    std::vector<int> Lw, Rw;
    for (int v : set) (X[3 * v + ax] <= cval ? Lw : Rw).push_back(v);
    if (Rw.empty()) {  // all on one side of the median plane: split by position
      Lw.assign(sorted.begin(), sorted.begin() + sorted.size() / 2);
      Rw.assign(sorted.begin() + sorted.size() / 2, sorted.end());
    }
    for (int v : Rw) side[v] = 2;
    std::vector<int> Ls, S;
    for (int v : Lw) {
      bool touches = false;
      for (int k = g->ptr[v]; k < g->ptr[v + 1] && !touches; ++k) touches = side[g->adj[k]] == 2;
      (touches ? S : Ls).push_back(v);
    }
    for (int v : Rw) side[v] = 0;
    if (Ls.empty() && Rw.size() == set.size() - S.size() && S.size() == set.size()) {
      throw std::runtime_error("nested dissection made no progress");
    }
    std::vector<int> top = run(std::move(Ls));
    std::vector<int> right = run(std::move(Rw));
    top.insert(top.end(), right.begin(), right.end());
    if (S.empty()) return top;
    seps.push_back(std::move(S));
    kids.push_back(std::move(top));
    return {(int)seps.size() - 1};
  }
};

}  // namespace

void build_layout(int nv, int ne, const double* X, const int32_t* tets, const uint8_t* pinned, int max_sub,
                  int levels, Layout& L) {
  L.nv = nv;
  L.ne = ne;
  Graph g = free_graph(nv, ne, tets, pinned);
  std::vector<int> free_set;
  for (int v = 0; v < nv; ++v)
    if (!pinned[v]) free_set.push_back(v);
  ND nd{X, &g, std::max(1, max_sub), std::vector<int>(nv, 0), {}, {}, {}};
  nd.run(free_set);

  // separator levels: 1 above subdomains only, else one more than the highest
  // separator below; the nodes at level >= `levels` become one top node
  const int no = (int)nd.seps.size();
  const int cap = levels > 0 ? levels : (1 << 30);
  std::vector<int> height(no, 1), oparent(no, -1);
  for (int o = 0; o < no; ++o)
    for (int c : nd.kids[o]) {
      height[o] = std::max(height[o], height[c] + 1);
      oparent[c] = o;
    }
  std::vector<int> order;  // unmerged nodes by (level, post-order)
  for (int o = 0; o < no; ++o)
    if (height[o] < cap) order.push_back(o);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return height[a] < height[b]; });
  std::vector<int> new_of(no, -1);
  for (int k = 0; k < (int)order.size(); ++k) new_of[order[k]] = k;
  const bool merged = (int)order.size() < no;
  const int n_nodes = (int)order.size() + (merged ? 1 : 0);
  for (int o = 0; o < no; ++o)
    if (height[o] >= cap) new_of[o] = n_nodes - 1;

  L.lib2orig.clear();
  L.sub_begin.clear();
  for (auto& s : nd.subs) {
    L.sub_begin.push_back((int)L.lib2orig.size());
    L.lib2orig.insert(L.lib2orig.end(), s.begin(), s.end());
  }
  L.nsub = (int)nd.subs.size();
  L.nB = (int)L.lib2orig.size();
  L.sub_begin.push_back(L.nB);
  L.sep_begin.assign(1, 0);
  L.sep_level.clear();
  L.sep_parent.clear();
  for (int k = 0; k < (int)order.size(); ++k) {
    const int o = order[k];
    L.lib2orig.insert(L.lib2orig.end(), nd.seps[o].begin(), nd.seps[o].end());
    L.sep_begin.push_back((int)L.lib2orig.size() - L.nB);
    L.sep_level.push_back(height[o]);
    L.sep_parent.push_back(oparent[o] < 0 ? -1 : new_of[oparent[o]]);
  }
  if (merged) {
    for (int o = 0; o < no; ++o)
      if (height[o] >= cap) L.lib2orig.insert(L.lib2orig.end(), nd.seps[o].begin(), nd.seps[o].end());
    L.sep_begin.push_back((int)L.lib2orig.size() - L.nB);
    L.sep_level.push_back(cap);
    L.sep_parent.push_back(-1);
  }
  L.nf = (int)L.lib2orig.size();
  L.nT = L.nf - L.nB;
  L.nlev = n_nodes ? L.sep_level.back() : 0;
  L.lev_begin.assign(L.nlev + 1, L.nT);
  for (int n = n_nodes - 1; n >= 0; --n) L.lev_begin[L.sep_level[n] - 1] = L.sep_begin[n];
  for (int l = L.nlev - 1; l >= 1; --l) L.lev_begin[l - 1] = std::min(L.lev_begin[l - 1], L.lev_begin[l]);
  for (int v = 0; v < nv; ++v)
    if (pinned[v]) L.lib2orig.push_back(v);
  L.orig2lib.assign(nv, -1);
  for (int i = 0; i < nv; ++i) L.orig2lib[L.lib2orig[i]] = i;

  // interface rows coupled to each subdomain; check the block structure
  std::vector<int> sub_of(nv, -1);
  for (int s = 0; s < L.nsub; ++s)
    for (int i = L.sub_begin[s]; i < L.sub_begin[s + 1]; ++i) sub_of[L.lib2orig[i]] = s;
  L.Irows.assign(L.nsub, {});
  for (int s = 0; s < L.nsub; ++s) {
    std::vector<int>& I = L.Irows[s];
    for (int i = L.sub_begin[s]; i < L.sub_begin[s + 1]; ++i) {
      int v = L.lib2orig[i];
      for (int k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
        int u = g.adj[k];
        int lu = L.orig2lib[u];
        if (sub_of[u] == s) continue;
        if (sub_of[u] >= 0 || lu < L.nB) throw std::runtime_error("subdomains are not separated");
        I.push_back(lu - L.nB);
      }
    }
    std::sort(I.begin(), I.end());
    I.erase(std::unique(I.begin(), I.end()), I.end());
  }

  // block structure of the separator tree: eliminating node n couples it to
  // the rows of higher levels that it touches through the mesh or through a
  // common subdomain, and to what its children's eliminations left there
  std::vector<int> node_of(L.nT);
  for (int n = 0; n < n_nodes; ++n)
    for (int i = L.sep_begin[n]; i < L.sep_begin[n + 1]; ++i) node_of[i] = n;
  std::vector<std::vector<int>> subs_of_row(L.nT);
  for (int s = 0; s < L.nsub; ++s)
    for (int p : L.Irows[s]) subs_of_row[p].push_back(s);
  std::vector<std::vector<int>> children(n_nodes);
  for (int n = 0; n < n_nodes; ++n)
    if (L.sep_parent[n] >= 0) children[L.sep_parent[n]].push_back(n);
  L.sep_struct.assign(n_nodes, {});
  std::vector<int> mark(L.nT, -1);
  for (int n = 0; n < n_nodes; ++n) {  // levels ascending: children first
    std::vector<int>& st = L.sep_struct[n];
    auto add = [&](int u) {
      if (node_of[u] == n || mark[u] == n) return;
      if (L.sep_level[node_of[u]] <= L.sep_level[n]) throw std::runtime_error("separator tree: coupled siblings");
      mark[u] = n;
      st.push_back(u);
    };
    for (int c : children[n])
      for (int u : L.sep_struct[c]) add(u);
    for (int i = L.sep_begin[n]; i < L.sep_begin[n + 1]; ++i) {
      const int v = L.lib2orig[L.nB + i];
      for (int k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
        const int u = L.orig2lib[g.adj[k]] - L.nB;
        if (u >= 0 && L.sep_level[node_of[u]] > L.sep_level[n]) add(u);
      }
      for (int s : subs_of_row[i])
        for (int u : L.Irows[s])
          if (L.sep_level[node_of[u]] > L.sep_level[n]) add(u);
    }
    std::sort(st.begin(), st.end());
  }

  // tets sorted by their smallest library vertex (locality of the gathers)
  std::vector<int> key(ne);
  for (int e = 0; e < ne; ++e) {
    int k = nv;
    for (int a = 0; a < 4; ++a) k = std::min(k, L.orig2lib[tets[4 * e + a]]);
    key[e] = k;
  }
  L.tet_lib2orig.resize(ne);
  std::iota(L.tet_lib2orig.begin(), L.tet_lib2orig.end(), 0);
  std::stable_sort(L.tet_lib2orig.begin(), L.tet_lib2orig.end(), [&](int a, int b) { return key[a] < key[b]; });
}

double factor_nnz_nd(int nv, int ne, const double* X, const int32_t* tets, const uint8_t* pinned) {
  Layout L;
  build_layout(nv, ne, X, tets, pinned, 16, 0, L);
  const int n = L.nf;
  Graph g = free_graph(nv, ne, tets, pinned);
  // adjacency in elimination order, lower part only (columns j < i of row i)
  std::vector<int> ptr(n + 1, 0), adj;
  adj.reserve(g.adj.size() / 2 + 1);
  for (int i = 0; i < n; ++i) {
    const int v = L.lib2orig[i];
    for (int k = g.ptr[v]; k < g.ptr[v + 1]; ++k) {
      const int j = L.orig2lib[g.adj[k]];
      if (j < i) adj.push_back(j);
    }
    ptr[i + 1] = (int)adj.size();
  }
  // elimination tree (with path compression through `anc`)
  std::vector<int> parent(n, -1), anc(n, -1);
  for (int i = 0; i < n; ++i)
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
      int r = adj[k];
      while (anc[r] != -1 && anc[r] != i) {
        const int t = anc[r];
        anc[r] = i;
        r = t;
      }
      if (anc[r] == -1) {
        anc[r] = i;
        parent[r] = i;
      }
    }
  // row counts: row i of L holds the etree nodes on the paths from the
  // columns of A's row i up to i
  std::vector<int> mark(n, -1);
  double nnz = n;
  for (int i = 0; i < n; ++i) {
    mark[i] = i;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k)
      for (int r = adj[k]; r != -1 && mark[r] != i; r = parent[r]) {
        mark[r] = i;
        nnz += 1.0;
      }
  }
  return nnz;
}

}  // namespace pdhot
