// Host-side tetrahedral mesh hierarchy and skeleton topology (Sec. 2 and
// Sec. 3.4.2 in three dimensions): faces, edges, edge patches with their
// colouring, Bey's red refinement and the averaging transfer at face
// centroids.
#pragma once
#include <string>
#include <vector>

namespace hdgmg {

struct Level3 {
  int nv = 0, nc = 0, nf = 0, nint = 0, ne = 0;
  std::vector<double> X;           // [nv][3]
  std::vector<int> cells;          // [nc][4] stored vertex order
  std::vector<int> faces;          // [nf][3] sorted vertex triples, lexicographic order
  std::vector<int> cell_faces;     // [nc][4] face opposite stored vertex i
  std::vector<int> face_cells;     // [nf][2] adjacent cells (-1 if none)
  std::vector<int> face_loc;       // [nf][2] local face index in those cells
  std::vector<int> int_id;         // [nf] interior number or -1
  std::vector<int> int_face;       // [nint] face of each interior number
  std::vector<double> fn, ft1, ft2;  // [nf][3] face frame n, t1, t2
  std::vector<double> farea;       // [nf]
  std::vector<double> vol;         // [nc]
  std::vector<int> sigma;          // [nc][4] n_{K,F} . n_F
  std::vector<int> parent;         // [nc] (levels > 0)
  std::vector<int> edges;          // [ne][2] sorted pairs, lexicographic order
  std::vector<int> cell_edges;     // [nc][6]
  std::vector<int> cell_dofs;      // [nc][4] interior face id or -1
  // edge (or vertex) patches with at least one interior face, colour-major
  // (edge or vertex order inside a colour)
  int ncol = 0;
  std::vector<int> colour_ptr;     // [ncol + 1]
  std::vector<int> patch_edge;     // [np]
  std::vector<int> pf_ptr, pf;     // patch -> interior face ids (ascending)
  std::vector<int> pc_ptr, pc;     // patch -> cells containing the edge
  int max_patch_faces = 0, max_patch_cells = 0;
};

// Skeleton of a tetrahedral mesh.  Returns "" or an error message.
std::string build_level3(Level3& L);

// Bey's red refinement: the midpoint of edge e becomes vertex nv + e; cell c
// = (x0,x1,x2,x3) has children 8c+0 (x0,x01,x02,x03), 8c+1 (x01,x1,x12,x13),
// 8c+2 (x02,x12,x2,x23), 8c+3 (x03,x13,x23,x3), 8c+4 (x01,x02,x03,x13),
// 8c+5 (x01,x02,x12,x13), 8c+6 (x02,x03,x13,x23), 8c+7 (x02,x12,x13,x23).
void refine3(const Level3& C, Level3& F);

// Edge patches and their greedy colouring: edges (with a non-empty patch)
// in edge order take the smallest colour unused by an earlier such edge
// sharing a cell, so that patches of one colour share no cell.
void build_edge_patches(Level3& L);

// Vertex patches (Sec. 3.4.2: the interior faces containing a vertex, the
// cells containing it) in the same fields (patch_edge then holds the
// vertex), greedily coloured in vertex order so that vertices of one colour
// lie in no common cell.
void build_vertex_patches(Level3& L);

// Averaging operator I_{l-1}^l (avgOpt) on the lowest-order unknowns (3 per
// interior face: n, t1, t2): the coarse CR field at the fine face centroid
// (the mean of the two sides on a coarse face), split in the fine face
// frame; sparse rows over fine unknowns.  inner[T][0..7]: the fine interior
// faces strictly inside coarse cell T (-1 padded).
struct Averaging3 {
  std::vector<int> row_ptr, col;
  std::vector<double> val;
  std::vector<int> inner;  // [nc_coarse][8]
};
void build_averaging3(const Level3& C, const Level3& F, Averaging3& A);

}  // namespace hdgmg
