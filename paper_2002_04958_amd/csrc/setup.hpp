// AMG setup on the device (natural ordering).
#pragma once
#include "common.hpp"

namespace mgd {

constexpr int8_t kC = 1, kF = -1, kU = 0;

struct SetupLevel {
  Csr<double> A;
  DBuf<int8_t> cf;  // empty on the coarsest level
  Csr<double> P;    // n x nc; empty on the coarsest level
  int nc = 0;
  int pmis_rounds = 0;
  DBuf<int> colour;  // Jones-Plassmann colours (multicolour Gauss-Seidel only)
  int ncolours = 0;
};

struct SetupHierarchy {
  std::vector<SetupLevel> levels;
  int coarse_kind = 0;           // 0 dense LU (explicit inverse), 1 l1-Jacobi sweeps
  DBuf<double> coarse_inv;       // n_L x n_L, column-major, when coarse_kind == 0
};

// Copy a caller matrix into an owned one.
void csr_copy_from(Ctx* c, const mgd_csr* A, Csr<double>& out);
void csr_copy(Ctx* c, const Csr<double>& A, Csr<double>& out);
// Build the hierarchy for a square matrix (already validated, copied in).
void amg_build(Ctx* c, Csr<double>&& A0, const amg_params& p, SetupHierarchy& H);

// Pieces exposed for testing and for the union builder.
void strength(Ctx* c, const Csr<double>& A, double theta, double dom, DBuf<uint8_t>& S,
              DBuf<int>& stc);
// hmis_tile > 0: HMIS with tiles of that many rows (<= 1024), else PMIS
int pmis(Ctx* c, const Csr<double>& A, const DBuf<uint8_t>& S, const DBuf<int>& stc,
         uint64_t seed, int level, DBuf<int8_t>& state, int hmis_tile);
void interpolation(Ctx* c, const Csr<double>& A, const DBuf<uint8_t>& S,
                   const DBuf<int8_t>& state, const DBuf<int>& cidx, int nc, Csr<double>& P);
// Sorted transpose (values copied).
void transpose(Ctx* c, const Csr<double>& A, Csr<double>& T);
// C = A B, structural pattern, entries summed over ascending k from 0.
void spgemm(Ctx* c, const Csr<double>& A, const Csr<double>& B, Csr<double>& C);
// d_i = a_ii + sum_{j != i} |a_ij| (ascending column order)
void l1_diagonal(Ctx* c, const Csr<double>& A, double* d);
// d_i = a_ii
void plain_diagonal(Ctx* c, const Csr<double>& A, double* d);
// Jones-Plassmann colouring of the structural graph of A; returns the number of colours
int jp_colouring(Ctx* c, const Csr<double>& A, uint64_t seed, int level, DBuf<int>& colour);
// Explicit inverse via LU with partial pivoting; returns false on a zero pivot.
bool dense_inverse(Ctx* c, const Csr<double>& A, DBuf<double>& inv_colmajor);

}  // namespace mgd
