// Mesh topology, element matrices, nested-dissection ordering and the
// supernodal symbolic structure, host C++.
#include "host_mesh.h"

#include <algorithm>
#include <cstring>
#include <stdexcept>

namespace tem {

static const int kAB[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};

void MeshTopo::init(int nx_, int ny_, int nz_) {
  nx = nx_;
  ny = ny_;
  nz = nz_;
  ex = (int64_t)nx * (ny + 1) * (nz + 1);
  ey = (int64_t)(nx + 1) * ny * (nz + 1);
  ez = (int64_t)(nx + 1) * (ny + 1) * nz;
  n_edges = ex + ey + ez;
  n_cells = (int64_t)nx * ny * nz;
  unk_of_edge.assign(n_edges, -1);
  edge_of_unk.clear();
  edge_of_unk.reserve(n_edges);
  int32_t u = 0;
  for (int64_t e = 0; e < n_edges; ++e) {
    int d, i, j, k;
    geometry(e, d, i, j, k);
    bool in;
    if (d == 0)
      in = (j > 0 && j < ny && k > 0 && k < nz);
    else if (d == 1)
      in = (i > 0 && i < nx && k > 0 && k < nz);
    else
      in = (i > 0 && i < nx && j > 0 && j < ny);
    if (in) {
      unk_of_edge[e] = u++;
      edge_of_unk.push_back((int32_t)e);
    }
  }
  n_unknowns = u;
  n_nodes = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  unk_of_node.assign(n_nodes, -1);
  node_of_unk.clear();
  int32_t v = 0;
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i)
        if (i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz) {
          unk_of_node[node(i, j, k)] = v++;
          node_of_unk.push_back((int32_t)node(i, j, k));
        }
  n_inodes = v;
}

void MeshTopo::geometry(int64_t e, int &dir, int &i, int &j, int &k) const {
  if (e < ex) {
    dir = 0;
    i = (int)(e % nx);
    int64_t r = e / nx;
    j = (int)(r % (ny + 1));
    k = (int)(r / (ny + 1));
    return;
  }
  e -= ex;
  if (e < ey) {
    dir = 1;
    i = (int)(e % (nx + 1));
    int64_t r = e / (nx + 1);
    j = (int)(r % ny);
    k = (int)(r / ny);
    return;
  }
  e -= ey;
  dir = 2;
  i = (int)(e % (nx + 1));
  int64_t r = e / (nx + 1);
  j = (int)(r % (ny + 1));
  k = (int)(r / (ny + 1));
}

void MeshTopo::cell_edges(int i, int j, int k, int64_t out[12]) const {
  for (int p = 0; p < 4; ++p) {
    int a = kAB[p][0], b = kAB[p][1];
    out[p] = xedge(i, j + a, k + b);
    out[4 + p] = yedge(i + a, j, k + b);
    out[8 + p] = zedge(i + a, j + b, k);
  }
}

// ---------------------------------------------------------------- elements
void element_mass_unit(double h, double out[144]) {
  // same-direction edges with transverse offsets (a,b),(a',b'):
  // h * m1[a][a'] * m1[b][b'], m1 = [[1/3,1/6],[1/6,1/3]]
  const double m1[2][2] = {{1.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 1.0 / 3.0}};
  std::memset(out, 0, sizeof(double) * 144);
  for (int d = 0; d < 3; ++d)
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < 4; ++q)
        out[(4 * d + p) * 12 + 4 * d + q] = h * m1[kAB[p][0]][kAB[q][0]] * m1[kAB[p][1]][kAB[q][1]];
}

void element_stiffness(double h, double mu, double out[144]) {
  // Stokes on each face: (curl E).n integrated = signed sum of edge DOFs.
  // Face f = 2*d + o (normal +d at offset o).  C[f][e] in {-1,0,1}.
  int C[6][12];
  std::memset(C, 0, sizeof(C));
  auto lx = [](int a, int b) { return a + 2 * b; };
  auto ly = [](int a, int b) { return 4 + a + 2 * b; };
  auto lz = [](int a, int b) { return 8 + a + 2 * b; };
  for (int o = 0; o < 2; ++o) {
    // x-face: dEz/dy - dEy/dz ; z-edges indexed (dx,dy), y-edges (dx,dz)
    C[o][lz(o, 1)] += 1;
    C[o][lz(o, 0)] -= 1;
    C[o][ly(o, 1)] -= 1;
    C[o][ly(o, 0)] += 1;
    // y-face: dEx/dz - dEz/dx ; x-edges (dy,dz), z-edges (dx,dy)
    C[2 + o][lx(o, 1)] += 1;
    C[2 + o][lx(o, 0)] -= 1;
    C[2 + o][lz(1, o)] -= 1;
    C[2 + o][lz(0, o)] += 1;
    // z-face: dEy/dx - dEx/dy ; y-edges (dx,dz), x-edges (dy,dz)
    C[4 + o][ly(1, o)] += 1;
    C[4 + o][ly(0, o)] -= 1;
    C[4 + o][lx(1, o)] -= 1;
    C[4 + o][lx(0, o)] += 1;
  }
  // face-function mass (unit flux functions): 1/(6h) [[2,1],[1,2]] per direction
  double Mf[6][6];
  std::memset(Mf, 0, sizeof(Mf));
  for (int d = 0; d < 3; ++d) {
    Mf[2 * d][2 * d] = Mf[2 * d + 1][2 * d + 1] = 2.0 / (6.0 * h);
    Mf[2 * d][2 * d + 1] = Mf[2 * d + 1][2 * d] = 1.0 / (6.0 * h);
  }
  for (int a = 0; a < 12; ++a)
    for (int b = 0; b < 12; ++b) {
      double s = 0.0;
      for (int f = 0; f < 6; ++f)
        for (int g = 0; g < 6; ++g) s += C[f][a] * Mf[f][g] * C[g][b];
      out[a * 12 + b] = s / mu;
    }
}

void element_gradient(int out[96]) {
  // edge (start node -> end node along +axis); local nodes (dx,dy,dz) -> dx + 2 dy + 4 dz
  std::memset(out, 0, sizeof(int) * 96);
  for (int p = 0; p < 4; ++p) {
    int a = kAB[p][0], b = kAB[p][1];
    // x-edge (dy=a, dz=b): (0,a,b) -> (1,a,b)
    out[p * 8 + (0 + 2 * a + 4 * b)] = -1;
    out[p * 8 + (1 + 2 * a + 4 * b)] = +1;
    // y-edge (dx=a, dz=b): (a,0,b) -> (a,1,b)
    out[(4 + p) * 8 + (a + 0 + 4 * b)] = -1;
    out[(4 + p) * 8 + (a + 2 + 4 * b)] = +1;
    // z-edge (dx=a, dy=b): (a,b,0) -> (a,b,1)
    out[(8 + p) * 8 + (a + 2 * b + 0)] = -1;
    out[(8 + p) * 8 + (a + 2 * b + 4)] = +1;
  }
}

void element_grad_mass(double h, double out[64]) {
  double M1[144];
  int G[96];
  element_mass_unit(h, M1);
  element_gradient(G);
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      double s = 0.0;
      for (int e = 0; e < 12; ++e)
        for (int f = 0; f < 12; ++f) s += G[e * 8 + a] * M1[e * 12 + f] * G[f * 8 + b];
      out[a * 8 + b] = s;
    }
}

// ------------------------------------------------------ nested dissection
namespace {

struct NDBuilder {
  const MeshTopo &mt;
  int leaf_max;
  Symbolic &sym;
  bool nodes;
  std::vector<int64_t> scratch;

  NDBuilder(const MeshTopo &m, int lm, Symbolic &s, bool nd) : mt(m), leaf_max(lm), sym(s), nodes(nd) {}

  // edges (nodes) in the closed box, not on its surface
  void interior(const int b[3][2], std::vector<int64_t> &out) {
    int x0 = b[0][0], x1 = b[0][1], y0 = b[1][0], y1 = b[1][1], z0 = b[2][0], z1 = b[2][1];
    if (nodes) {
      for (int k = z0 + 1; k < z1; ++k)
        for (int j = y0 + 1; j < y1; ++j)
          for (int i = x0 + 1; i < x1; ++i) out.push_back(mt.node(i, j, k));
      return;
    }
    for (int k = z0 + 1; k < z1; ++k)
      for (int j = y0 + 1; j < y1; ++j)
        for (int i = x0; i < x1; ++i) out.push_back(mt.xedge(i, j, k));
    for (int k = z0 + 1; k < z1; ++k)
      for (int j = y0; j < y1; ++j)
        for (int i = x0 + 1; i < x1; ++i) out.push_back(mt.yedge(i, j, k));
    for (int k = z0; k < z1; ++k)
      for (int j = y0 + 1; j < y1; ++j)
        for (int i = x0 + 1; i < x1; ++i) out.push_back(mt.zedge(i, j, k));
  }

  // edges (nodes) in the plane {axis = p} inside the closed box, not on its surface
  void plane(const int b[3][2], int axis, int p, std::vector<int64_t> &out) {
    int x0 = b[0][0], x1 = b[0][1], y0 = b[1][0], y1 = b[1][1], z0 = b[2][0], z1 = b[2][1];
    if (nodes) {
      if (axis == 0) {
        for (int k = z0 + 1; k < z1; ++k)
          for (int j = y0 + 1; j < y1; ++j) out.push_back(mt.node(p, j, k));
      } else if (axis == 1) {
        for (int k = z0 + 1; k < z1; ++k)
          for (int i = x0 + 1; i < x1; ++i) out.push_back(mt.node(i, p, k));
      } else {
        for (int j = y0 + 1; j < y1; ++j)
          for (int i = x0 + 1; i < x1; ++i) out.push_back(mt.node(i, j, p));
      }
      return;
    }
    if (axis == 0) {
      for (int k = z0 + 1; k < z1; ++k)
        for (int j = y0; j < y1; ++j) out.push_back(mt.yedge(p, j, k));
      for (int k = z0; k < z1; ++k)
        for (int j = y0 + 1; j < y1; ++j) out.push_back(mt.zedge(p, j, k));
    } else if (axis == 1) {
      for (int k = z0 + 1; k < z1; ++k)
        for (int i = x0; i < x1; ++i) out.push_back(mt.xedge(i, p, k));
      for (int k = z0; k < z1; ++k)
        for (int i = x0 + 1; i < x1; ++i) out.push_back(mt.zedge(i, p, k));
    } else {
      for (int j = y0 + 1; j < y1; ++j)
        for (int i = x0; i < x1; ++i) out.push_back(mt.xedge(i, j, p));
      for (int j = y0; j < y1; ++j)
        for (int i = x0 + 1; i < x1; ++i) out.push_back(mt.yedge(i, j, p));
    }
  }

  void emit_cols(std::vector<int64_t> &edges, SymNode &nd) {
    std::sort(edges.begin(), edges.end());
    nd.first = (int64_t)sym.perm.size();
    for (int64_t e : edges) {
      int32_t u = nodes ? mt.unk_of_node[e] : mt.unk_of_edge[e];
      if (u < 0) throw std::runtime_error("nested dissection produced a boundary entity");
      sym.perm.push_back(u);
    }
    nd.last = (int64_t)sym.perm.size();
  }

  int rec(const int b[3][2], int level) {
    int side[3] = {b[0][1] - b[0][0], b[1][1] - b[1][0], b[2][1] - b[2][0]};
    int mx = std::max(side[0], std::max(side[1], side[2]));
    SymNode nd;
    std::memcpy(nd.box, b, sizeof(nd.box));
    nd.level = level;
    if (mx <= leaf_max) {
      scratch.clear();
      interior(b, scratch);
      emit_cols(scratch, nd);
      nd.sub_first = nd.first;
      sym.nodes.push_back(nd);
      return (int)sym.nodes.size() - 1;
    }
    int axis = 0;
    if (side[1] > side[axis]) axis = 1;
    if (side[2] > side[axis]) axis = 2;
    int lo = b[axis][0], hi = b[axis][1];
    int p = lo + (hi - lo) / 2;
    int b1[3][2], b2[3][2];
    std::memcpy(b1, b, sizeof(b1));
    std::memcpy(b2, b, sizeof(b2));
    b1[axis][1] = p;
    b2[axis][0] = p;
    int c1 = rec(b1, level + 1);
    int c2 = rec(b2, level + 1);
    scratch.clear();
    plane(b, axis, p, scratch);
    emit_cols(scratch, nd);
    nd.child[0] = c1;
    nd.child[1] = c2;
    nd.sub_first = sym.nodes[c1].sub_first;
    sym.nodes.push_back(nd);
    int me = (int)sym.nodes.size() - 1;
    sym.nodes[c1].parent = me;
    sym.nodes[c2].parent = me;
    return me;
  }
};

// cells that contain canonical edge e, with the edge's local index
int edge_cells(const MeshTopo &mt, int64_t e, int cells[4][3], int local[4]) {
  int d, i, j, k;
  mt.geometry(e, d, i, j, k);
  int n = 0;
  for (int p = 0; p < 4; ++p) {
    int a = kAB[p][0], b = kAB[p][1];
    int ci, cj, ck;
    if (d == 0) {
      ci = i; cj = j - a; ck = k - b;
    } else if (d == 1) {
      ci = i - a; cj = j; ck = k - b;
    } else {
      ci = i - a; cj = j - b; ck = k;
    }
    if (ci < 0 || cj < 0 || ck < 0 || ci >= mt.nx || cj >= mt.ny || ck >= mt.nz) continue;
    cells[n][0] = ci;
    cells[n][1] = cj;
    cells[n][2] = ck;
    local[n] = 4 * d + p;
    ++n;
  }
  return n;
}

// cells that contain canonical node v
int node_cells(const MeshTopo &mt, int64_t v, int cells[8][3]) {
  int i = (int)(v % (mt.nx + 1));
  int64_t r = v / (mt.nx + 1);
  int j = (int)(r % (mt.ny + 1)), k = (int)(r / (mt.ny + 1));
  int n = 0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        int ci = i - dx, cj = j - dy, ck = k - dz;
        if (ci < 0 || cj < 0 || ck < 0 || ci >= mt.nx || cj >= mt.ny || ck >= mt.nz) continue;
        cells[n][0] = ci;
        cells[n][1] = cj;
        cells[n][2] = ck;
        ++n;
      }
  return n;
}

// unknown indices of the entities sharing a cell with canonical entity x
void neighbours(const MeshTopo &mt, bool nodes, int64_t x, std::vector<int32_t> &out) {
  out.clear();
  if (nodes) {
    int cells[8][3];
    int nc = node_cells(mt, x, cells);
    for (int c = 0; c < nc; ++c)
      for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            int32_t u = mt.unk_of_node[mt.node(cells[c][0] + dx, cells[c][1] + dy, cells[c][2] + dz)];
            if (u >= 0) out.push_back(u);
          }
    return;
  }
  int cells[4][3], local[4];
  int64_t ce[12];
  int nc = edge_cells(mt, x, cells, local);
  for (int c = 0; c < nc; ++c) {
    mt.cell_edges(cells[c][0], cells[c][1], cells[c][2], ce);
    for (int b = 0; b < 12; ++b) {
      int32_t u = mt.unk_of_edge[ce[b]];
      if (u >= 0) out.push_back(u);
    }
  }
}

}  // namespace

void analyse_symbolic(const MeshTopo &mt, int leaf_max, Symbolic &sym, bool nodes) {
  sym = Symbolic();
  sym.leaf_max = leaf_max;
  const int64_t N = nodes ? mt.n_inodes : mt.n_unknowns;
  sym.perm.reserve(N);
  NDBuilder nb(mt, leaf_max, sym, nodes);
  int root[3][2] = {{0, mt.nx}, {0, mt.ny}, {0, mt.nz}};
  nb.rec(root, 0);
  if ((int64_t)sym.perm.size() != N) throw std::runtime_error("ordering does not cover all unknowns");
  sym.iperm.assign(N, -1);
  for (int64_t q = 0; q < N; ++q) sym.iperm[sym.perm[q]] = (int32_t)q;
  // U_s = (adj(cols(s)) U children's U) \ [sub_first, last)
  std::vector<int32_t> cand, nb_;
  sym.rows.clear();
  for (size_t s = 0; s < sym.nodes.size(); ++s) {
    SymNode &nd = sym.nodes[s];
    cand.clear();
    for (int64_t q = nd.first; q < nd.last; ++q) {
      int64_t x = nodes ? mt.node_of_unk[sym.perm[q]] : mt.edge_of_unk[sym.perm[q]];
      neighbours(mt, nodes, x, nb_);
      for (int32_t u : nb_) {
        int32_t r = sym.iperm[u];
        if (r < nd.sub_first || r >= nd.last) cand.push_back(r);
      }
    }
    for (int c = 0; c < 2; ++c) {
      if (nd.child[c] < 0) continue;
      const SymNode &ch = sym.nodes[nd.child[c]];
      for (int64_t a = 0; a < ch.nrows; ++a) {
        int32_t r = sym.rows[ch.rows_off + a];
        if (r < nd.sub_first || r >= nd.last) cand.push_back(r);
      }
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
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
    double k = (double)(nd.last - nd.first), u = (double)nd.nrows;
    sym.max_front = std::max(sym.max_front, (int)(nd.last - nd.first + nd.nrows));
    sym.flops_per_pole += 8.0 * ((k + u) * (k + u) * (k + u) - u * u * u) / 6.0;
    sym.nnz_l += (nd.last - nd.first) * (nd.last - nd.first + 1) / 2 + (nd.last - nd.first) * nd.nrows;
  }
}

void build_pattern(const MeshTopo &mt, const std::vector<int32_t> &perm, Pattern &pat,
                   bool nodes) {
  const int64_t N = nodes ? mt.n_inodes : mt.n_unknowns;
  std::vector<int32_t> iperm(N);
  for (int64_t q = 0; q < N; ++q) iperm[perm[q]] = (int32_t)q;
  pat.row_edge.resize(N);
  pat.edge_new.assign(nodes ? mt.n_nodes : mt.n_edges, -1);
  for (int64_t q = 0; q < N; ++q) {
    int32_t e = nodes ? mt.node_of_unk[perm[q]] : mt.edge_of_unk[perm[q]];
    pat.row_edge[q] = e;
    pat.edge_new[e] = (int32_t)q;
  }
  pat.rowptr.assign(N + 1, 0);
  pat.col.clear();
  pat.col.reserve(N * (nodes ? 27 : 33));
  std::vector<int32_t> buf, nb_;
  for (int64_t q = 0; q < N; ++q) {
    buf.clear();
    neighbours(mt, nodes, pat.row_edge[q], nb_);
    for (int32_t u : nb_) buf.push_back(iperm[u]);
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    pat.col.insert(pat.col.end(), buf.begin(), buf.end());
    pat.rowptr[q + 1] = (int64_t)pat.col.size();
  }
}

}  // namespace tem
