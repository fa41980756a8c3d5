// Host-side numeric setup: quadrature tables, the harmonic-extension
// intergrid transfers of the lowest-order hierarchy and the coarsest-level
// inverse (FP64).  Runs once per assemble.
#pragma once
#include <vector>

#include "element.hpp"
#include "topology.hpp"

namespace hdgmg {

struct CSR {
  int n = 0;  // rows
  std::vector<int> rp, ci;
  std::vector<double> v;
};

// Stroud data rule with k+2 points per direction and the facet Gauss rule.
QuadTables make_tables(int k);

// Convection rules of order k (see ConvTables).
ConvTables make_conv_tables(int k);

// Viscosity of every level: the finest as given (one value per cell), each
// coarser cell the mean of its four children.
void level_viscosities(const std::vector<Level>& lv, const std::vector<double>& nu_fine,
                       std::vector<std::vector<double>>& nu);

// Closed-form lowest-order cell blocks of a level, [nc][6][6].
void host_cr_blocks(const Level& L, const std::vector<double>& nu, double beta, double eps_inv,
                    std::vector<double>& B);

// Stabilised transfer (id - E_T A_TT^-1 A_T.) I from coarse level C to its
// refinement F (div-transfer, harmonic-ex) as CSR over fine DOFs, for the
// fine operator with cell blocks B ([nc][6][6] row-major; transpose: use
// the blocks' transposes, i.e. the operator A^T).  general: the interior
// blocks may be nonsymmetric (LU instead of Cholesky).  False if an interior
// block is singular.
bool stabilised_transfer(const Level& C, const Level& F, const Averaging& Av, const std::vector<double>& B,
                         bool transpose, bool general, CSR& P);

// Transpose of a CSR matrix with ncols columns.
void csr_transpose(const CSR& A, int ncols, CSR& T);

// Assembled lowest-order operator of a level from its cell blocks, as CSR
// over the 2 n_int unknowns (columns sorted).
void assemble_csr(const Level& L, const std::vector<double>& B, CSR& A);

// Column-major inverse of the assembled coarsest operator A^eps_{0,1} with
// cell blocks B0 (general: LU instead of Cholesky).
bool coarse_inverse(const Level& L0, const std::vector<double>& B0, bool general, std::vector<double>& inv);

// Cholesky-based inverse of a dense SPD matrix (row-major in, column-major out).
bool invert_spd(const std::vector<double>& A, int n, std::vector<double>& inv);

// LU (partial pivoting) inverse of a dense matrix (row-major in, column-major out).
bool invert_general(const std::vector<double>& A, int n, std::vector<double>& inv);

}  // namespace hdgmg
