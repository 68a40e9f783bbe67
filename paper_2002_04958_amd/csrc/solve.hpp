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
#include <map>
#include <memory>

#include "common.hpp"
#include "setup.hpp"

namespace mgd {

struct DenseDev {
  int off;  // natural offset at this level
  int n;
  const double* inv;  // column-major n x n
};

template <typename T>
struct ULevel {
  int n = 0;         // natural rows (including dense-solved members)
  int nS = 0;        // stored rows
  int nC = 0;        // C-block size
  int n_coarse = 0;  // rows of level l+1 (0: no coarser level)
  long long nnz_S_C = 0, nnz_S_F = 0;
  Csr<T> A;          // nS rows, natural columns
  DBuf<int> perm;    // stored -> natural
  DBuf<T> dinv;      // 1 / l1 diagonal, per stored row
  Csr<T> W;          // nS - nC rows, n_coarse columns
  Csr<T> Wt;         // n_coarse rows, nS - nC columns
  int tpr = 1, tpr_w = 1, tpr_wt = 1;
  std::vector<DenseDev> dense;
  DBuf<DenseDev> dense_dev;
  int dense_max_n = 0;
  long long dense_entries = 0;
};

template <typename T>
struct Union {
  std::vector<ULevel<T>> L;
  std::vector<DBuf<T>> b, X0, X1, r;  // per level (b[0], X1[0] unused: caller's)
  DBuf<T> t0, t1;                     // finest-level scratch for extra cycles
  int n0 = 0;
  int n_pre = 1, n_post = 1;
  int members = 0;

  // z = k V-cycles on b (zero initial guess); b, z natural level-0 vectors.
  void apply(Ctx* c, const T* b, T* z, int cycles);
  void vcycle(Ctx* c, const T* b, T* z);
  double bytes_per_vcycle() const;
};

template <typename T>
std::unique_ptr<Union<T>> build_union(Ctx* c, const std::vector<const SetupHierarchy*>& members,
                                      int n_pre, int n_post, int autotune);

// Tuned row-group widths, keyed by (rows, nnz, max row length); persisted to
// the JSON file named by MGD_AUTOTUNE_CACHE when set.
int autotune_lookup(long long rows, long long nnz, int maxrow, bool fp32);
void autotune_store(long long rows, long long nnz, int maxrow, bool fp32, int tpr);

}  // namespace mgd
