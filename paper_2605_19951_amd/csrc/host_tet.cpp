// Tetrahedral mesh topology, the RT0 mass diagonal and the nested
// dissection of a general graph, host C++.
#include <algorithm>
#include <array>
#include <cstring>
#include <cmath>
#include <numeric>
#include <stdexcept>

#include "host_mesh.h"

namespace tem {

namespace {

const int kLE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

double det3(const double a[3], const double b[3], const double c[3]) {
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
         a[2] * (b[0] * c[1] - b[1] * c[0]);
}

}  // namespace

std::string TetTopo::init(const double *x, const int32_t *t, int64_t nn, int64_t nt) {
  if (nn < 4 || nt < 1) return "a tetrahedral mesh needs at least 4 nodes and 1 tetrahedron";
  if (nn > ((int64_t)1 << 31) - 1 || nt > ((int64_t)1 << 29))
    return "tetrahedral mesh too large for 32-bit ids";
  n_nodes = nn;
  n_tets = nt;
  xyz.assign(x, x + 3 * nn);
  tets.assign(t, t + 4 * nt);
  for (double v : xyz)
    if (!std::isfinite(v)) return "node coordinates must be finite";
  for (int64_t c = 0; c < nt; ++c) {
    const int32_t *q = &tets[4 * c];
    for (int i = 0; i < 4; ++i) {
      if (q[i] < 0 || q[i] >= nn) return "tetrahedron node id out of range";
      for (int j = 0; j < i; ++j)
        if (q[i] == q[j]) return "tetrahedron with a repeated node";
    }
    double e[3][3], len = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 3; ++d) {
        e[i][d] = xyz[3 * q[i + 1] + d] - xyz[3 * q[0] + d];
        len = std::max(len, std::fabs(e[i][d]));
      }
    if (!(std::fabs(det3(e[0], e[1], e[2])) > 1e-12 * len * len * len))
      return "degenerate tetrahedron (zero volume)";
  }
  // canonical edges
  std::vector<int64_t> keys((size_t)nt * 6);
  for (int64_t c = 0; c < nt; ++c)
    for (int l = 0; l < 6; ++l) {
      int64_t a = tets[4 * c + kLE[l][0]], b = tets[4 * c + kLE[l][1]];
      if (a > b) std::swap(a, b);
      keys[c * 6 + l] = a * nn + b;
    }
  std::vector<int64_t> ek(keys);
  std::sort(ek.begin(), ek.end());
  ek.erase(std::unique(ek.begin(), ek.end()), ek.end());
  n_edges = (int64_t)ek.size();
  if (n_edges > ((int64_t)1 << 31) - 1) return "too many edges for 32-bit ids";
  edges.resize(2 * n_edges);
  for (int64_t e = 0; e < n_edges; ++e) {
    edges[2 * e] = (int32_t)(ek[e] / nn);
    edges[2 * e + 1] = (int32_t)(ek[e] % nn);
  }
  auto edge_of = [&](int64_t a, int64_t b) {
    if (a > b) std::swap(a, b);
    return (int64_t)(std::lower_bound(ek.begin(), ek.end(), a * nn + b) - ek.begin());
  };
  tet_edges.resize((size_t)nt * 6);
  tet_signs.resize((size_t)nt * 6);
  for (int64_t c = 0; c < nt; ++c)
    for (int l = 0; l < 6; ++l) {
      tet_edges[c * 6 + l] = (int32_t)(std::lower_bound(ek.begin(), ek.end(), keys[c * 6 + l]) - ek.begin());
      tet_signs[c * 6 + l] = tets[4 * c + kLE[l][0]] < tets[4 * c + kLE[l][1]] ? 1 : -1;
    }
  // faces: (sorted triple, tetrahedron, opposite local node)
  struct F {
    std::array<int32_t, 3> v;
    int32_t tet;
    int8_t opp;
  };
  std::vector<F> fs((size_t)nt * 4);
  for (int64_t c = 0; c < nt; ++c)
    for (int p = 0; p < 4; ++p) {
      F f;
      int k = 0;
      for (int i = 0; i < 4; ++i)
        if (i != p) f.v[k++] = tets[4 * c + i];
      std::sort(f.v.begin(), f.v.end());
      f.tet = (int32_t)c;
      f.opp = (int8_t)p;
      fs[c * 4 + p] = f;
    }
  std::sort(fs.begin(), fs.end(), [](const F &a, const F &b) {
    return a.v != b.v ? a.v < b.v : a.tet < b.tet;
  });
  std::vector<char> bnd(n_edges, 0), bnode(nn, 0);
  iface_tets.clear();
  iface_opp.clear();
  for (size_t i = 0; i < fs.size();) {
    size_t j = i;
    while (j < fs.size() && fs[j].v == fs[i].v) ++j;
    if (j - i > 2) return "non-conforming mesh: a face shared by more than two tetrahedra";
    if (j - i == 1) {
      const auto &v = fs[i].v;
      bnd[edge_of(v[0], v[1])] = 1;
      bnd[edge_of(v[0], v[2])] = 1;
      bnd[edge_of(v[1], v[2])] = 1;
      bnode[v[0]] = bnode[v[1]] = bnode[v[2]] = 1;
    } else {
      iface_tets.push_back(fs[i].tet);
      iface_tets.push_back(fs[i + 1].tet);
      iface_opp.push_back(fs[i].opp);
      iface_opp.push_back(fs[i + 1].opp);
    }
    i = j;
  }
  unk_of_edge.assign(n_edges, -1);
  edge_of_unk.clear();
  for (int64_t e = 0; e < n_edges; ++e)
    if (!bnd[e]) {
      unk_of_edge[e] = (int32_t)edge_of_unk.size();
      edge_of_unk.push_back((int32_t)e);
    }
  n_unknowns = (int64_t)edge_of_unk.size();
  unk_of_node.assign(nn, -1);
  node_of_unk.clear();
  for (int64_t v = 0; v < nn; ++v)
    if (!bnode[v]) {
      unk_of_node[v] = (int32_t)node_of_unk.size();
      node_of_unk.push_back((int32_t)v);
    }
  n_inodes = (int64_t)node_of_unk.size();
  {
    std::vector<int64_t> nc(n_inodes + 1, 0);
    for (int64_t c = 0; c < nt; ++c) {
      int ni = 0;
      for (int i = 0; i < 4; ++i) ni += unk_of_node[tets[4 * c + i]] >= 0;
      for (int i = 0; i < 4; ++i) {
        const int32_t u = unk_of_node[tets[4 * c + i]];
        if (u >= 0) nc[u + 1] += ni;
      }
    }
    for (int64_t u = 0; u < n_inodes; ++u) nc[u + 1] += nc[u];
    std::vector<int32_t> raw(nc[n_inodes]);
    std::vector<int64_t> fill(nc.begin(), nc.end() - 1);
    for (int64_t c = 0; c < nt; ++c)
      for (int i = 0; i < 4; ++i) {
        const int32_t u = unk_of_node[tets[4 * c + i]];
        if (u < 0) continue;
        for (int j = 0; j < 4; ++j) {
          const int32_t w = unk_of_node[tets[4 * c + j]];
          if (w >= 0) raw[fill[u]++] = w;
        }
      }
    nadj_ptr.assign(n_inodes + 1, 0);
    nadj.clear();
    for (int64_t u = 0; u < n_inodes; ++u) {
      std::sort(raw.begin() + nc[u], raw.begin() + nc[u + 1]);
      auto end = std::unique(raw.begin() + nc[u], raw.begin() + nc[u + 1]);
      nadj.insert(nadj.end(), raw.begin() + nc[u], end);
      nadj_ptr[u + 1] = (int64_t)nadj.size();
    }
  }
  // unknown adjacency through shared tetrahedra
  std::vector<int64_t> cnt(n_unknowns + 1, 0);
  for (int64_t c = 0; c < nt; ++c) {
    int nu = 0;
    for (int l = 0; l < 6; ++l) nu += unk_of_edge[tet_edges[c * 6 + l]] >= 0;
    for (int l = 0; l < 6; ++l) {
      const int32_t u = unk_of_edge[tet_edges[c * 6 + l]];
      if (u >= 0) cnt[u + 1] += nu;
    }
  }
  for (int64_t u = 0; u < n_unknowns; ++u) cnt[u + 1] += cnt[u];
  std::vector<int32_t> raw(cnt[n_unknowns]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t c = 0; c < nt; ++c)
    for (int l = 0; l < 6; ++l) {
      const int32_t u = unk_of_edge[tet_edges[c * 6 + l]];
      if (u < 0) continue;
      for (int m = 0; m < 6; ++m) {
        const int32_t w = unk_of_edge[tet_edges[c * 6 + m]];
        if (w >= 0) raw[fill[u]++] = w;
      }
    }
  adj_ptr.assign(n_unknowns + 1, 0);
  adj.clear();
  adj.reserve(raw.size() / 2);
  for (int64_t u = 0; u < n_unknowns; ++u) {
    std::sort(raw.begin() + cnt[u], raw.begin() + cnt[u + 1]);
    auto end = std::unique(raw.begin() + cnt[u], raw.begin() + cnt[u + 1]);
    adj.insert(adj.end(), raw.begin() + cnt[u], end);
    adj_ptr[u + 1] = (int64_t)adj.size();
  }
  return "";
}

// Face function of the face opposite node p: (x - x_p) / (3 |T|) (unit
// flux); its squared norm is (int |x - c|^2 + |T| |c - x_p|^2) / (9 |T|^2)
// with c the centroid and int (x - c)(x - c)^T = |T| / 20 sum_i (x_i - c)(x_i - c)^T.
void tet_rt0_diag(const double x[12], double out[4]) {
  double e[3][3];
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) e[i][d] = x[3 * (i + 1) + d] - x[d];
  const double vol = std::fabs(det3(e[0], e[1], e[2])) / 6.0;
  double c[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i)
    for (int d = 0; d < 3; ++d) c[d] += 0.25 * x[3 * i + d];
  double tr = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int d = 0; d < 3; ++d) tr += (x[3 * i + d] - c[d]) * (x[3 * i + d] - c[d]);
  const double second = vol / 20.0 * tr;
  for (int p = 0; p < 4; ++p) {
    double dd = 0.0;
    for (int d = 0; d < 3; ++d) dd += (c[d] - x[3 * p + d]) * (c[d] - x[3 * p + d]);
    out[p] = (second + vol * dd) / (9.0 * vol * vol);
  }
}

namespace {

struct GraphND {
  const std::vector<int64_t> &ap;
  const std::vector<int32_t> &aj;
  const std::vector<double> &xy;
  int64_t leaf_max;
  Symbolic &sym;
  std::vector<int8_t> side;

  void emit(std::vector<int32_t> &cols, SymNode &nd) {
    std::sort(cols.begin(), cols.end());
    nd.first = (int64_t)sym.perm.size();
    sym.perm.insert(sym.perm.end(), cols.begin(), cols.end());
    nd.last = (int64_t)sym.perm.size();
  }

  int leaf(std::vector<int32_t> &V, int level) {
    SymNode nd;
    std::memset(nd.box, 0, sizeof(nd.box));
    nd.level = level;
    emit(V, nd);
    nd.sub_first = nd.first;
    sym.nodes.push_back(nd);
    return (int)sym.nodes.size() - 1;
  }

  // Smallest vertex separator inside the two one-sided boundaries: a
  // minimum vertex cover of the bipartite graph of the cut edges between SA
  // and SB (Hopcroft-Karp matching, then Konig's construction: Z = vertices
  // reached from unmatched SA vertices by alternating paths, cover =
  // (SA \ Z) + (SB & Z)).  Uncovered boundary vertices go back to their side.
  // side[] still marks A (1) and B (2) on entry.
  std::vector<int32_t> loc;

  void min_cover(const std::vector<int32_t> &SA, const std::vector<int32_t> &SB,
                 std::vector<int32_t> &A, std::vector<int32_t> &B, std::vector<int32_t> &S) {
    const int L = (int)SA.size(), R = (int)SB.size();
    if (loc.empty()) loc.assign(side.size(), -1);
    for (int i = 0; i < L; ++i) loc[SA[i]] = i;
    for (int j = 0; j < R; ++j) loc[SB[j]] = j;
    std::vector<int64_t> gp(L + 1, 0);
    std::vector<int32_t> gj;
    for (int i = 0; i < L; ++i) {
      const int32_t v = SA[i];
      for (int64_t t = ap[v]; t < ap[v + 1]; ++t)
        if (side[aj[t]] == 2) gj.push_back(loc[aj[t]]);
      gp[i + 1] = (int64_t)gj.size();
    }
    std::vector<int> mL(L, -1), mR(R, -1), dist(L), it(L);
    const int INF = 1 << 30;
    std::vector<int> q;
    q.reserve(L);
    auto bfs = [&]() {
      q.clear();
      bool found = false;
      for (int i = 0; i < L; ++i) {
        dist[i] = mL[i] < 0 ? 0 : INF;
        if (mL[i] < 0) q.push_back(i);
      }
      for (size_t h = 0; h < q.size(); ++h) {
        const int u = q[h];
        for (int64_t t = gp[u]; t < gp[u + 1]; ++t) {
          const int w = mR[gj[t]];
          if (w < 0)
            found = true;
          else if (dist[w] == INF) {
            dist[w] = dist[u] + 1;
            q.push_back(w);
          }
        }
      }
      return found;
    };
    // iterative layered DFS for an augmenting path from free vertex u0
    std::vector<int> stk;
    auto dfs = [&](int u0) {
      stk.assign(1, u0);
      while (!stk.empty()) {
        const int u = stk.back();
        bool advanced = false;
        for (; it[u] < gp[u + 1] - gp[u]; ++it[u]) {
          const int r = gj[gp[u] + it[u]], w = mR[r];
          if (w < 0) {   // augment along the stack
            for (int k = (int)stk.size() - 1; k >= 0; --k) {
              const int uu = stk[k], rr = gj[gp[uu] + it[uu]];
              mL[uu] = rr;
              mR[rr] = uu;
            }
            return true;
          }
          if (dist[w] == dist[u] + 1) {
            stk.push_back(w);
            advanced = true;
            break;
          }
        }
        if (!advanced) {
          dist[u] = INF;
          stk.pop_back();
          if (!stk.empty()) ++it[stk.back()];
        }
      }
      return false;
    };
    while (bfs()) {
      std::fill(it.begin(), it.end(), 0);
      for (int i = 0; i < L; ++i)
        if (mL[i] < 0) dfs(i);
    }
    // Konig: alternating reachability from the unmatched left vertices
    std::vector<char> zl(L, 0), zr(R, 0);
    q.clear();
    for (int i = 0; i < L; ++i)
      if (mL[i] < 0) {
        zl[i] = 1;
        q.push_back(i);
      }
    for (size_t h = 0; h < q.size(); ++h) {
      const int u = q[h];
      for (int64_t t = gp[u]; t < gp[u + 1]; ++t) {
        const int r = gj[t];
        if (zr[r] || mL[u] == r) continue;
        zr[r] = 1;
        const int w = mR[r];
        if (w >= 0 && !zl[w]) {
          zl[w] = 1;
          q.push_back(w);
        }
      }
    }
    for (int i = 0; i < L; ++i) (zl[i] ? A : S).push_back(SA[i]);
    for (int j = 0; j < R; ++j) (zr[j] ? S : B).push_back(SB[j]);
    for (int32_t v : SA) loc[v] = -1;
    for (int32_t v : SB) loc[v] = -1;
  }

  int rec(std::vector<int32_t> &V, int level) {
    if ((int64_t)V.size() <= leaf_max) return leaf(V, level);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t v : V)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], xy[3 * (size_t)v + d]);
        hi[d] = std::max(hi[d], xy[3 * (size_t)v + d]);
      }
    int axis = 0;
    for (int d = 1; d < 3; ++d)
      if (hi[d] - lo[d] > hi[axis] - lo[axis]) axis = d;
    const size_t h = V.size() / 2;
    std::nth_element(V.begin(), V.begin() + h, V.end(), [&](int32_t a, int32_t b) {
      const double xa = xy[3 * (size_t)a + axis], xb = xy[3 * (size_t)b + axis];
      return xa != xb ? xa < xb : a < b;
    });
    for (size_t i = 0; i < V.size(); ++i) side[V[i]] = i < h ? 1 : 2;
    std::vector<int32_t> A, B, SA, SB;
    for (size_t i = 0; i < V.size(); ++i) {
      const int32_t v = V[i];
      const int8_t me = side[v], other = me == 1 ? 2 : 1;
      bool cut = false;
      for (int64_t t = ap[v]; t < ap[v + 1] && !cut; ++t) cut = side[aj[t]] == other;
      if (me == 1)
        (cut ? SA : A).push_back(v);
      else
        (cut ? SB : B).push_back(v);
    }
    std::vector<int32_t> S;
    min_cover(SA, SB, A, B, S);
    for (int32_t v : V) side[v] = 0;
    if (S.empty()) {   // the halves are not connected: a one-vertex separator
      std::vector<int32_t> &big = A.size() >= B.size() ? A : B;
      S.push_back(big.back());
      big.pop_back();
    }
    if (A.empty() || B.empty()) return leaf(V, level);
    std::vector<int32_t>().swap(V);
    const int c1 = rec(A, level + 1);
    const int c2 = rec(B, level + 1);
    SymNode nd;
    std::memset(nd.box, 0, sizeof(nd.box));
    nd.level = level;
    emit(S, nd);
    nd.child[0] = c1;
    nd.child[1] = c2;
    nd.sub_first = sym.nodes[c1].sub_first;
    sym.nodes.push_back(nd);
    const int me = (int)sym.nodes.size() - 1;
    sym.nodes[c1].parent = me;
    sym.nodes[c2].parent = me;
    return me;
  }
};

}  // namespace

void analyse_graph(int64_t n, const std::vector<int64_t> &adj_ptr, const std::vector<int32_t> &adj,
                   const std::vector<double> &coords, int64_t leaf_max, Symbolic &sym) {
  sym = Symbolic();
  sym.leaf_max = (int)std::min<int64_t>(leaf_max, 1 << 30);
  sym.perm.reserve(n);
  if (n > 0) {
    GraphND g{adj_ptr, adj, coords, std::max<int64_t>(leaf_max, 1), sym, std::vector<int8_t>(n, 0)};
    std::vector<int32_t> all(n);
    std::iota(all.begin(), all.end(), 0);
    g.rec(all, 0);
  }
  if ((int64_t)sym.perm.size() != n) throw std::runtime_error("ordering does not cover all unknowns");
  sym.iperm.assign(n, -1);
  for (int64_t q = 0; q < n; ++q) sym.iperm[sym.perm[q]] = (int32_t)q;
  // levels by depth were set during the recursion; U_s = (adj(cols(s)) U
  // children's U) \ [sub_first, last), all of it later than s
  std::vector<int32_t> cand;
  for (size_t s = 0; s < sym.nodes.size(); ++s) {
    SymNode &nd = sym.nodes[s];
    cand.clear();
    for (int64_t q = nd.first; q < nd.last; ++q) {
      const int32_t v = sym.perm[q];
      for (int64_t t = adj_ptr[v]; t < adj_ptr[v + 1]; ++t) {
        const int32_t r = sym.iperm[adj[t]];
        if (r < nd.sub_first || r >= nd.last) cand.push_back(r);
      }
    }
    for (int c = 0; c < 2; ++c) {
      if (nd.child[c] < 0) continue;
      const SymNode &ch = sym.nodes[nd.child[c]];
      for (int64_t a = 0; a < ch.nrows; ++a) {
        const int32_t r = sym.rows[ch.rows_off + a];
        if (r < nd.sub_first || r >= nd.last) cand.push_back(r);
      }
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    if (!cand.empty() && cand.front() < nd.last)
      throw std::runtime_error("nested dissection left a coupling to an earlier subtree");
    nd.rows_off = (int64_t)sym.rows.size();
    nd.nrows = (int64_t)cand.size();
    sym.rows.insert(sym.rows.end(), cand.begin(), cand.end());
  }
  sym.n_levels = 0;
  sym.max_front = 0;
  sym.flops_per_pole = 0.0;
  sym.nnz_l = 0;
  for (const SymNode &nd : sym.nodes) {
    sym.n_levels = std::max(sym.n_levels, nd.level + 1);
    const double k = (double)(nd.last - nd.first), u = (double)nd.nrows;
    sym.max_front = std::max(sym.max_front, (int)(nd.last - nd.first + nd.nrows));
    sym.flops_per_pole += 8.0 * ((k + u) * (k + u) * (k + u) - u * u * u) / 6.0;
    sym.nnz_l += (nd.last - nd.first) * (nd.last - nd.first + 1) / 2 + (nd.last - nd.first) * nd.nrows;
  }
}

void build_pattern_graph(const std::vector<int64_t> &adj_ptr, const std::vector<int32_t> &adj,
                         const std::vector<int32_t> &perm, const std::vector<int32_t> &ent_of_vertex,
                         int64_t n_ent, Pattern &pat) {
  const int64_t N = (int64_t)perm.size();
  std::vector<int32_t> iperm(N);
  for (int64_t q = 0; q < N; ++q) iperm[perm[q]] = (int32_t)q;
  pat.row_edge.resize(N);
  pat.edge_new.assign(n_ent, -1);
  for (int64_t q = 0; q < N; ++q) {
    const int32_t e = ent_of_vertex[perm[q]];
    pat.row_edge[q] = e;
    pat.edge_new[e] = (int32_t)q;
  }
  pat.rowptr.assign(N + 1, 0);
  pat.col.clear();
  pat.col.reserve(adj.size());
  std::vector<int32_t> buf;
  for (int64_t q = 0; q < N; ++q) {
    const int32_t v = perm[q];
    buf.clear();
    for (int64_t t = adj_ptr[v]; t < adj_ptr[v + 1]; ++t) buf.push_back(iperm[adj[t]]);
    std::sort(buf.begin(), buf.end());
    pat.col.insert(pat.col.end(), buf.begin(), buf.end());
    pat.rowptr[q + 1] = (int64_t)pat.col.size();
  }
}

}  // namespace tem
