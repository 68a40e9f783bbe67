// Solve-phase V-cycle over a union of one or more AMG hierarchies.
//
// Level l of a union concatenates level l of every member hierarchy that has
// one, in member order ("natural" union numbering: member offsets, each
// member's own row order).  Rows are STORED C-block first (every coarsening
// member's C points, in member order and ascending index), then the F-block
// (F points, and every row of a member whose last level is relaxed rather
// than solved).  Members whose last level is solved densely keep their rows
// out of the stored matrix and are handled by the dense solve kernel.
// Because coarse points are numbered in ascending fine order, the C-block
// position of a C point IS its coarse index, so P = [I; W] and R = [I, W^T]
// with only W and W^T stored.  Columns stay in natural numbering, so vectors
// are never permuted.
#pragma once
#include <array>
#include <map>
#include <memory>

#include "common.hpp"
#include "setup.hpp"

namespace mgd {

// one member's input of a batched apply, read from a block vector of
// (G+2) segments of N rows
struct SegIn {
  int seg;              // source segment of the Krylov vector (0..G+1)
  const double* coef;   // subtract coef o w (or nullptr)
};

struct DenseDev {
  int off;  // first row of the member in the level's extended stored order
  int n;
  const double* inv;  // column-major n x n
};

// A level matrix in one of two layouts chosen per level:
//   SELL: slices of 64 consecutive rows, each stored column-major with the
//         slice's longest row as its width (entry e of row 64 s + t at
//         off[s] + 64 e + t; padding entries are zero with the row's own
//         column), so one lane per row reads consecutive addresses;
//   SELL16: SELL with 16-bit column offsets (below);
//   CSR:  row pointers, and `tpr` lanes of a wavefront per row.
template <typename T>
struct LMat {
  int rows = 0, fmt = 0, tpr = 1;  // fmt: 0 CSR, 1 SELL, 2 SELL16
  int bs = 256;                    // threads per workgroup of the kernels reading it
  long long nnz = 0;               // entries (without padding)
  long long stored = 0;            // stored entries (with padding)
  DBuf<int> rp;                    // CSR: rows + 1 row pointers; SELL: slices + 1 offsets;
                                   // SELL16: 4 slices + 2 (offsets, two column bases)
  DBuf<int> ci;                    // SELL16: 16-bit codes, two per element
  DBuf<T> v;
};
// SELL16: SELL whose columns are 16-bit offsets from two bases per slice,
// one for the columns below a split (the C-block of a level matrix) and one
// for the rest (bit 15 set).  A slice whose columns on either side of the
// split span 2^15 or more (the slice across the C/F boundary of a union)
// keeps 32-bit columns.  Slice s keeps at rp[4s .. 4s+3] the offset of its
// values, the offset of its column codes in 16-bit units (even), the C base
// and the F base (-1: 32-bit columns); rp[4 * slices] and rp[4 * slices + 1]
// hold the totals.
enum { kFmtCSR = 0, kFmtSELL = 1, kFmtSELL16 = 2 };

// One level of a union in extended stored order: [0, nC) the C-block, [nC, nS)
// the F-block (rows smoothed, F points and relaxed coarsest rows), [nS, nX)
// rows of members solved densely at this level.  Every vector of the level is
// kept in this order; columns of A are stored-order indices.
template <typename T>
struct ULevel {
  int n = 0;          // rows (== nX)
  int nS = 0, nC = 0; // stored rows, C-block size
  int nX = 0;         // extended rows
  int nX_next = 0;    // rows of level l+1 (0: last level)
  int nC_next = 0, nS_next = 0;
  long long nnz_C = 0, nnz_F = 0;  // entries of C rows and of F rows
  LMat<T> A;          // nS rows, stored-order columns
  DBuf<T> dinv;       // 1 / l1 diagonal, stored rows
  DBuf<int> perm;     // extended stored order -> natural union numbering (nX)
  DBuf<int> iperm;    // level 0: natural union numbering -> extended stored order
  DBuf<T> dinv_nat;   // level 0: dinv at the natural position of each C row, else 0
  LMat<T> W;          // F rows of P (nS - nC rows), columns in level l+1 extended order
  LMat<T> Wt;         // W transposed, rows in level l+1 extended order, columns F index
  DBuf<int> cmap;     // C row I -> its level l+1 extended index (nC)
  DBuf<int> cpos;     // level l+1 extended index k -> C row of this level (nX_next)
  DBuf<T> dgs;        // 1 / a_ii (multicolour Gauss-Seidel)
  std::vector<std::array<int, 4>> cranges;  // per colour: C-block [lo, hi), F-block [lo, hi)
  std::vector<DenseDev> dense;
  DBuf<DenseDev> dense_dev;
  int dense_max_n = 0;
  long long dense_entries = 0;
};

// One phase of the persistent tail: the small levels of a V-cycle run in one
// launch, phase after phase, separated by a grid-wide barrier.  Each phase is
// one of the per-level launches below with the same arguments.
enum : int { kTopFHalf0 = 0, kTopHalf = 1, kTopResid = 2, kTopRestrict = 3, kTopProlong = 4,
             kTopDense = 5 };
template <typename T>
struct TailOp {
  int kind, fmt, tpr;
  int r0, r1;                 // rows of the phase
  int nC, nS;                 // C-block (and stored rows) of the gathered level
  int nCn, pre;               // restrict: next level's C-block, first-sweep C values;
                              // prolong: this level's C-block
  long long f_minus_c, d_minus_c;
  const int* rp;              // matrix (A, W^T or W): read only
  const int* ci;
  const T* v;
  const T* dinv;              // 1 / d of the rows (restrict: of the next level)
  const T* B;                 // right-hand side (restrict: the residual)
  const T* xc;                // gathered vector, buffer of its C region
  const T* xold;              // half-sweep: previous values of the rows
  T* out;                     // rows written
  T* out2;                    // restrict: next level's C values; prolong: C region
  const int* map;             // restrict: cpos; prolong: cmap
  const DenseDev* dense;      // dense solves: members, 64-row chunks per member
  int ndense, dchunks;
};

// A union's level-0 result left in stored order: member m's row i sits at
// stored index k = iperm[m N + i] of the C region (k < nC), the F region
// (k < nS) or the dense rows (each region in a buffer of its own, indexed by k)
template <typename T>
struct StoredOut {
  const int* iperm;
  const T *xc, *xf, *xd;
  int nC, nS;
};

template <typename T>
struct Union {
  std::vector<ULevel<T>> L;
  // per level: right-hand side (nX), two iterate buffers (nX; the C and F
  // regions alternate between them independently), residual (nS)
  std::vector<DBuf<T>> B, X0, X1, R;
  DBuf<T> t1;  // natural level-0 scratch for extra cycles
  int n0 = 0;
  int n_pre = 1, n_post = 1;
  int members = 0;
  bool gs = false;  // multicolour Gauss-Seidel instead of CF-l1-Jacobi

  // persistent tail: levels >= tail_from run as one launch of tail_blocks
  // workgroups over the phase table tail_ops (tail_from < 0: no tail)
  int tail_from = -1, tail_nops = 0, tail_blocks = 0;
  int tail_cc = 0, tail_cf = 0;  // iterate buffers of level tail_from after the tail
  double tail_bytes = 0, tail_bytes_csr = 0;
  DBuf<TailOp<T>> tail_ops;
  DBuf<unsigned> tail_sync;  // barrier counters (reset by the last workgroup out)
  void build_tail(Ctx* c);

  // z = k V-cycles on b (zero initial guess); b, z natural level-0 vectors.
  void apply(Ctx* c, const T* b, T* z, int cycles);
  // One cycle with the members' right-hand sides formed in the entry kernel:
  // member m's is (T)(r[tab[m].seg] - tab[m].coef o w) over N rows, the same
  // arithmetic as forming them into a vector first and calling apply.
  // With z null (CF-l1-Jacobi only) the result stays in stored order, the
  // final C half-sweep in place, for stored_out() to read until the next cycle.
  void apply_seg(Ctx* c, int N, const SegIn* tab, const double* r, const T* w, T* z);
  StoredOut<T> stored_out() const;
  double bytes_per_vcycle() const;

 private:
  int out_cc = 0, out_cf = 0;  // level-0 buffers of the C and F regions after a cycle
  // one V-cycle on B[0] (already in stored order, C values of X0[0] set)
  // ending with z (natural) = the result, or with it left in stored order (z null)
  void vcycle(Ctx* c, T* z);
  void vcycle_gs(Ctx* c, T* z);
  void gs_sweep(Ctx* c, int l, bool descending);
};

template <typename T>
std::unique_ptr<Union<T>> build_union(Ctx* c, const std::vector<const SetupHierarchy*>& members,
                                      int n_pre, int n_post, int autotune, int smoother);

// Tuned layouts, keyed by the matrix's role (kind: "" a level matrix, "wt:" a
// restriction) and (rows, nnz, max row length); persisted to the JSON file
// named by MGD_AUTOTUNE_CACHE when set.
int autotune_lookup(long long rows, long long nnz, int maxrow, bool fp32, const char* kind = "");
// Level kernels' row ranges per workgroup: contiguous shares per chiplet (1)
// or in dispatch order (0) for every device kernel launched afterwards.
void set_xcd_rows(int on);
void autotune_store(long long rows, long long nnz, int maxrow, bool fp32, int tpr,
                    const char* kind = "");

}  // namespace mgd
