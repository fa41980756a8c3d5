// Host-side mesh hierarchy and skeleton topology (Sec. 2, Sec. 3.4.2).
//
// Built once per context on the host from the coarse mesh; everything here
// is integer topology or geometric weights that the device kernels consume.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hdgmg {

struct Level {
  int nv = 0, nc = 0, nf = 0, nint = 0;
  std::vector<double> X;          // [nv][2]
  std::vector<int> cells;         // [nc][3] stored vertex order
  std::vector<int> edges;         // [nf][2], v0 < v1, lexicographic order
  std::vector<int> cell_facets;   // [nc][3], facet opposite local vertex i
  std::vector<int> facet_cells;   // [nf][2] adjacent cells (-1 if none)
  std::vector<int> facet_loc;     // [nf][2] local facet index in that cell
  // do-nothing (outflow) facets: input vertex pairs (sorted), then a flag
  // per facet; they carry unknowns and are numbered with the interior ones
  std::vector<std::pair<int, int>> outflow_in;
  std::vector<char> outflow;      // [nf]
  std::vector<int> int_id;        // [nf] unknown-carrying (interior or do-nothing) number, or -1
  std::vector<int> int_facet;     // [nint] facet of each such number
  std::vector<double> tang, norm; // [nf][2] facet frame
  std::vector<double> len;        // [nf]
  std::vector<double> area;       // [nc]
  std::vector<int> sigma;         // [nc][3] n_{K,F} . n_F
  std::vector<int> parent;        // [nc] (levels > 0)
  // vertex-patch smoother data
  std::vector<int> colour;        // [nv]
  int ncol = 0;
  std::vector<int> colour_ptr;    // [ncol+1] ranges of patches
  std::vector<int> patch_vertex;  // [np] patch -> vertex (colour-major)
  std::vector<int> patch_facet_ptr, patch_facets;  // CSR, interior ids sorted
  std::vector<int> patch_cell_ptr, patch_cells;    // CSR, cells at the vertex
  int max_patch_facets = 0;
  // cell -> interior facet ids (-1 on the boundary): [nc][3]
  std::vector<int> cell_dofs;
};

// Build the skeleton of a triangulation.  Returns "" or an error message.
std::string build_level(Level& L);

// Red refinement with the canonical numbering (see hdgmg.h).
void refine(const Level& C, Level& F);

// Canonical vertex colouring and the patch lists.
void build_patches(Level& L);

// Edge (facet) patches in the same fields: each unknown-carrying facet
// alone (patch_vertex then holds the facet), greedily coloured in facet
// order so that facets of one colour lie in no common cell.
void build_facet_patches(Level& L);

// Averaging operator I_{l-1}^l (avgOpt) on the lowest-order unknowns
// (2 per interior facet: normal, tangential), as sparse rows: for fine
// DOF r, entries (coarse DOF, weight).  Also the fine DOFs strictly inside
// each coarse cell (6 per coarse cell, or fewer when a fine facet is on the
// boundary, which cannot happen for interior middle-triangle facets).
struct Averaging {
  std::vector<int> row_ptr, col;   // CSR over fine DOFs
  std::vector<double> val;
  std::vector<int> inner_facets;   // [nc_coarse][3] fine interior ids
};
void build_averaging(const Level& C, const Level& F, Averaging& A);

}  // namespace hdgmg
