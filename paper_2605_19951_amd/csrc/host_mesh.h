// Host-side mesh topology, element matrices and the supernodal symbolic
// structure of the shifted matrices A_i = K - xi_i M (one structure for all
// poles).  Pure C++; no HIP types, so it also builds into the host-only
// symbolic entry point.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace tem {

struct MeshTopo {
  int nx = 0, ny = 0, nz = 0;
  int64_t ex = 0, ey = 0, ez = 0, n_edges = 0, n_cells = 0;
  std::vector<int32_t> unk_of_edge;   // canonical edge -> unknown index or -1
  std::vector<int32_t> edge_of_unk;   // unknown index -> canonical edge
  int64_t n_unknowns = 0;
  // interior nodes (the nodal functions whose gradients span the null space
  // of the curl-curl operator with tangential-E boundary condition)
  int64_t n_nodes = 0;
  std::vector<int32_t> unk_of_node;   // canonical node -> interior index or -1
  std::vector<int32_t> node_of_unk;
  int64_t n_inodes = 0;
  int64_t node(int i, int j, int k) const { return i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k); }

  void init(int nx_, int ny_, int nz_);
  int64_t xedge(int i, int j, int k) const { return i + (int64_t)nx * (j + (int64_t)(ny + 1) * k); }
  int64_t yedge(int i, int j, int k) const { return ex + i + (int64_t)(nx + 1) * (j + (int64_t)ny * k); }
  int64_t zedge(int i, int j, int k) const {
    return ex + ey + i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k);
  }
  // direction and lower node of a canonical edge
  void geometry(int64_t e, int &dir, int &i, int &j, int &k) const;
  // the 12 edges of cell (i,j,k) in local order: x-edges (dy,dz), y-edges
  // (dx,dz), z-edges (dx,dy), each over (0,0),(1,0),(0,1),(1,1)
  void cell_edges(int i, int j, int k, int64_t out[12]) const;
};

// 12x12 element matrices (row-major): unit-conductivity mass and stiffness.
void element_mass_unit(double h, double out[144]);
void element_stiffness(double h, double mu, double out[144]);
// 8x8 nodal matrix G_c^T M1_c G_c of one cell (unit conductivity); local
// node order (dx,dy,dz) = (0,0,0),(1,0,0),(0,1,0),(1,1,0),(0,0,1),...
void element_grad_mass(double h, double out[64]);
// local gradient of one cell: 12 edges x 8 nodes, entries -1/0/+1
void element_gradient(int out[96]);

struct SymNode {
  int box[3][2];
  int64_t first = 0, last = 0;   // column range (new indices)
  int64_t sub_first = 0;         // first new index of the subtree
  int parent = -1;
  int child[2] = {-1, -1};
  int level = 0;                 // depth, root = 0
  int64_t rows_off = 0;          // U_s = rows[rows_off .. rows_off + nrows)
  int64_t nrows = 0;
};

struct Symbolic {
  int leaf_max = 4;
  std::vector<SymNode> nodes;          // post-order
  std::vector<int32_t> perm;           // new -> unknown
  std::vector<int32_t> iperm;          // unknown -> new
  std::vector<int32_t> rows;           // concatenated U_s (new indices)
  int n_levels = 0;
  int max_front = 0;
  double flops_per_pole = 0.0;
  int64_t nnz_l = 0;
};

// Nested dissection + supernodal symbolic factorisation (exact spec of the
// ordering: longest side split at lo + (hi-lo)/2, ties x < y < z, leaves of
// side <= leaf_max, post-order numbering, columns by canonical id).
// Unknowns are the interior edges; with `nodes` the interior nodes (same
// boxes, separators = nodes of the split plane inside the box).
void analyse_symbolic(const MeshTopo &mt, int leaf_max, Symbolic &sym, bool nodes = false);

// CSR pattern of "shares a cell" between unknowns, in the ordering given by
// perm (perm[new] = unknown); columns sorted.  row_edge[new] = canonical edge.
struct Pattern {
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<int32_t> row_edge;   // canonical edge (or node) of each row
  std::vector<int32_t> edge_new;   // canonical edge (or node) -> new index or -1
};
void build_pattern(const MeshTopo &mt, const std::vector<int32_t> &perm, Pattern &pat,
                   bool nodes = false);

}  // namespace tem

namespace tem {

// Tetrahedral mesh topology.  Canonical edges are the distinct node pairs
// (a, b), a < b, sorted lexicographically and oriented a -> b; the unknowns
// are the edges on no boundary face (a face of one tetrahedron only), in
// canonical order.
struct TetTopo {
  int64_t n_nodes = 0, n_tets = 0, n_edges = 0, n_unknowns = 0;
  std::vector<double> xyz;           // 3 per node
  std::vector<int32_t> tets;         // 4 per tetrahedron
  std::vector<int32_t> edges;        // 2 per canonical edge
  std::vector<int32_t> tet_edges;    // 6 per tetrahedron, local edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)
  std::vector<int8_t> tet_signs;     // +1 where the local direction i -> j is the canonical one
  std::vector<int32_t> unk_of_edge;  // canonical edge -> unknown or -1
  std::vector<int32_t> edge_of_unk;
  // faces shared by two tetrahedra: the two tetrahedra and, for each, the
  // local index of the node opposite the face
  std::vector<int32_t> iface_tets;   // 2 per interior face
  std::vector<int8_t> iface_opp;     // 2 per interior face
  // unknown adjacency (unknowns sharing a tetrahedron, itself included), CSR
  // in unknown order with sorted columns
  std::vector<int64_t> adj_ptr;
  std::vector<int32_t> adj;
  // interior nodes (on no boundary face; their hat functions' gradients
  // span the curl-free part of the unknown space) and their adjacency
  // (interior nodes sharing a tetrahedron, itself included)
  int64_t n_inodes = 0;
  std::vector<int32_t> unk_of_node, node_of_unk;
  std::vector<int64_t> nadj_ptr;
  std::vector<int32_t> nadj;
  // Build from host arrays; returns an error text ("" on success).
  std::string init(const double *xyz, const int32_t *tets, int64_t n_nodes, int64_t n_tets);
};

// Diagonal of the 4x4 lowest-order Raviart-Thomas mass matrix of one
// tetrahedron (x: 12 coordinates), face functions of unit flux, the face
// opposite local node p first-to-last.
void tet_rt0_diag(const double x[12], double out[4]);

// Nested dissection of a graph with vertex coordinates and the supernodal
// symbolic factorisation (the separator of each split is one supernode).
// Each subgraph of more than leaf_max vertices is split at the median of its
// longest coordinate extent; the separator is a minimum vertex cover of the
// edges the split cuts (it lies in the two sets of vertices with a
// neighbour on the other side).  Columns within a
// supernode are in increasing vertex order; supernodes in post-order.
//   adj_ptr/adj: symmetric adjacency (self loops allowed), coords: 3 per vertex.
void analyse_graph(int64_t n, const std::vector<int64_t> &adj_ptr, const std::vector<int32_t> &adj,
                   const std::vector<double> &coords, int64_t leaf_max, Symbolic &sym);

// CSR pattern of the adjacency in the ordering perm (perm[new] = vertex);
// row_edge[new] = canonical id of the vertex (ent_of_vertex), edge_new maps
// canonical ids (n_ent of them) to new indices or -1.
void build_pattern_graph(const std::vector<int64_t> &adj_ptr, const std::vector<int32_t> &adj,
                         const std::vector<int32_t> &perm, const std::vector<int32_t> &ent_of_vertex,
                         int64_t n_ent, Pattern &pat);

}  // namespace tem
