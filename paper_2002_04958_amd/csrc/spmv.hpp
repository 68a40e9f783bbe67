// Device-side description of the block system of eq. 2.2.
#pragma once
#include "common.hpp"

namespace mgd {

constexpr int kMaxBlocks = 66;  // G + 2 <= 66

struct BlockCsr {
  const int* rp;
  const int* ci;
  const double* v;
};

// Half storage of a shared-pattern system whose every block equals its
// transpose bit for bit (the assembled diffusion blocks): per block, the
// values on and above the diagonal of each row, row after row (sym_urp: N + 1
// row starts); per pattern entry, the position of its value there (sym_src:
// its own on and above the diagonal, its mirror's (j, i) below).  Rows hold at
// most kSymMaxRow entries, at most kSymMaxUpper of them on and above the
// diagonal (the 2D and 3D stencils).
constexpr int kSymMaxRow = 7;
constexpr int kSymMaxUpper = 4;

// Passed by value as a kernel argument.
struct BlockSysDev {
  int G, N;
  int tpr;
  int shared;  // 1: every block uses blk[0].rp / blk[0].ci (one pattern)
  int sym;     // 1: the half storage below is set (shared pattern only)
  BlockCsr blk[kMaxBlocks];
  long long nnz[kMaxBlocks];
  const double* d_gE;
  const double* d_Eg;
  const double* d_EI;
  const double* d_IE;
  const int* sym_urp;
  const int* sym_src;
  long long sym_nnz;  // half-storage entries per block
  const double* sym_v[kMaxBlocks];
};

BlockSysDev make_block_sys_dev(const mgd_block_system* A);
// Sets S's half storage when A is a library-owned system (assembled or
// transposed) whose blocks are symmetric; MGD_SYM_MATVEC=0 turns it off.
void attach_half_storage(const mgd_block_system* A, BlockSysDev& S);
void check_block_system(const mgd_block_system* A);
// y = A x, or y = b - A x when b != nullptr.
void block_matvec(Ctx* c, const BlockSysDev& S, const double* x, const double* b, double* y);
double block_matvec_bytes(const BlockSysDev& S, bool resid, bool csr);
// y = A x in two parts (shared pattern only): the part that does not read x_E,
// on `stream`, and, on the context stream once x_E is known, the rest; the
// result equals block_matvec's bit for bit.
void block_matvec_split(Ctx* c, const BlockSysDev& S, const double* x, double* y,
                        hipStream_t stream);
void block_matvec_finish(Ctx* c, const BlockSysDev& S, const double* x, double* y);

}  // namespace mgd
