// CSR SpMV and the block matvec of eq. 2.2.
#include "kernels.hpp"
#include "rowdot.hpp"
#include "spmv.hpp"

namespace mgd {

template <int TPR>
__global__ void __launch_bounds__(256) k_spmv(int n, const int* __restrict__ rp,
                                              const int* __restrict__ ci,
                                              const double* __restrict__ v,
                                              const double* __restrict__ x,
                                              double* __restrict__ y) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int row = (int)(t / TPR);
  const int lane = (int)(t % TPR);
  if (row >= n) return;
  double s = row_dot<TPR, double>(rp, ci, v, x, row, lane);
  if (lane == 0) y[row] = s;
}

template <int TPR>
struct SpmvLaunch {
  static void run(Ctx* c, const CsrView<double>& A, const double* x, double* y) {
    int grid = cdiv((long long)A.n_rows * TPR, 256);
    hipLaunchKernelGGL(k_spmv<TPR>, dim3(grid), dim3(256), 0, c->stream, A.n_rows, A.rp, A.ci, A.v,
                       x, y);
    MGD_CHECK_LAUNCH();
  }
};

void spmv(Ctx* c, const CsrView<double>& A, const double* x, double* y, int tpr, int cls) {
  if (A.n_rows == 0) return;
  ProfScope ps(c, cls, 12.0 * A.nnz + 4.0 * (A.n_rows + 1) + 8.0 * A.n_rows + 8.0 * A.n_cols,
               ksym(c, "k_spmv", {std::to_string(tpr_of(tpr))}));
  dispatch_tpr<SpmvLaunch>(tpr, c, A, x, y);
}

// ---------------------------------------------------------------------------
// Block matvec of eq. 2.2 over all (G+2) N rows in one launch:
//   y_g = A_g x_g + d_gE o x_E
//   y_E = A_E x_E + sum_g d_Eg[g] o x_g + d_EI o x_I
//   y_I = A_I x_I + d_IE o x_E
// (RESID: y = b - A x instead).  blockIdx.y selects the block.
// ---------------------------------------------------------------------------
template <int TPR, bool RESID>
__global__ void __launch_bounds__(256) k_block_matvec(BlockSysDev S, const double* __restrict__ x,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ y) {
  const int a = blockIdx.y;
  const int G = S.G, N = S.N;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int i = (int)(t / TPR);
  const int lane = (int)(t % TPR);
  if (i >= N) return;
  const BlockCsr B = S.blk[a];
  const double* xa = x + (size_t)a * N;
  double s = row_dot<TPR, double>(B.rp, B.ci, B.v, xa, i, lane);
  if (lane != 0) return;
  const double* xE = x + (size_t)G * N;
  if (a < G) {
    s += S.d_gE[(size_t)a * N + i] * xE[i];
  } else if (a == G) {
    for (int g = 0; g < G; ++g) s += S.d_Eg[(size_t)g * N + i] * x[(size_t)g * N + i];
    s += S.d_EI[i] * x[(size_t)(G + 1) * N + i];
  } else {
    s += S.d_IE[i] * xE[i];
  }
  const size_t r = (size_t)a * N + i;
  y[r] = RESID ? b[r] - s : s;
}

template <int TPR>
struct BlockMatvecLaunch {
  static void run(Ctx* c, const BlockSysDev& S, const double* x, const double* b, double* y) {
    dim3 grid(cdiv((long long)S.N * TPR, 256), S.G + 2);
    if (b)
      hipLaunchKernelGGL((k_block_matvec<TPR, true>), grid, dim3(256), 0, c->stream, S, x, b, y);
    else
      hipLaunchKernelGGL((k_block_matvec<TPR, false>), grid, dim3(256), 0, c->stream, S, x, b, y);
    MGD_CHECK_LAUNCH();
  }
};

// ---------------------------------------------------------------------------
// Block matvec of eq. 2.2 when every block has the same sparsity pattern (the
// assembled stencil, and its transpose).  A workgroup takes R consecutive
// rows of all G+2 blocks.  It stages the pattern segment of those rows (row
// pointers and column indices) in LDS once; then, block after block, every
// thread issues all of its coalesced loads of the block's values for the
// segment into registers before the barrier, the values go to LDS, and each
// thread sums its own row over its entries in stored order.  The column
// indices are read from HBM once per matvec instead of once per block.  A
// segment longer than the LDS capacity is walked in chunks, re-staging the
// column indices per chunk.  The E row's coupling sum  sum_g d_Eg[g] o x_g
// is accumulated while the thread passes block g, where x_g[i] was just
// gathered.
// ---------------------------------------------------------------------------
//
// SPLIT: the part that does not read x_E, for overlap with the work that
// produces x_E: y_g = A_g x_g, y_I = A_I x_I and y_E = sum_g d_Eg[g] o x_g
// (the E block's values are not read); k_block_matvec_finish adds the rest
// in the order of the whole kernel, so that the result is the same.
//
// SYM (S.sym: every block equal to its transpose, rows of at most kSymMaxRow
// entries): a block's values are read from its half storage.  The segment of
// the workgroup's rows (on and above the diagonal) is staged in LDS; an entry
// below the diagonal takes its mirror's value, from LDS when the mirror row is
// one of the workgroup's rows, else from the half storage in memory.  The
// values are the same bits, summed in the same order, so the result is that
// of the full storage; the values move about 4/7 of the bytes (3D stencil).
template <int R, bool RESID, bool SPLIT, bool SYM>
__global__ void __launch_bounds__(R, (SYM && !SPLIT) ? 4 : 1) k_block_matvec_shared(BlockSysDev S,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ y) {
  constexpr int CAP = 7 * R + 64;        // staged pattern entries per chunk
  constexpr int PT = (CAP + R - 1) / R;  // staging loads per thread and block
  static_assert(!SYM || kSymMaxRow * R <= CAP, "a symmetric segment must fit one chunk");
  // SYM: a half-storage segment holds at most kSymMaxUpper values per row
  constexpr int VCAP = SYM ? kSymMaxUpper * R : CAP;
  __shared__ int s_rp[R + 1];
  __shared__ int s_ci[CAP];
  __shared__ double s_v[VCAP];
  __shared__ int s_src[SYM ? kSymMaxRow * R : 1];
  const int G = S.G, N = S.N, nb = S.G + 2;
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * R;
  const int nr = min(R, N - i0);
  const int* __restrict__ rp = S.blk[0].rp;
  const int* __restrict__ ci = S.blk[0].ci;
  for (int k = t; k <= nr; k += R) s_rp[k] = rp[i0 + k];
  __syncthreads();
  const int beg = s_rp[0], end = s_rp[nr];
  const bool active = t < nr;
  const int i = i0 + t;
  const int rb = active ? s_rp[t] : 0, re = active ? s_rp[t + 1] : 0;
  const bool one_chunk = end - beg <= CAP;  // always with SYM (rows of <= kSymMaxRow)
  if (one_chunk)
    for (int k = t; k < end - beg; k += R) {
      s_ci[k] = ci[beg + k];
      if (SYM) s_src[k] = S.sym_src[beg + k];
    }
  // SYM: the half-storage segment [ub, ue) of the workgroup's rows, and the
  // thread's row (at most kSymMaxRow entries): columns and value positions,
  // the same for every block, kept in registers
  const int ub = SYM ? S.sym_urp[i0] : 0, ue = SYM ? S.sym_urp[i0 + nr] : 0;
  int sj[kSymMaxRow], su[kSymMaxRow];
  const int ne = SYM ? re - rb : 0;
  if (SYM) {
    __syncthreads();  // s_ci and s_src staged
#pragma unroll
    for (int q = 0; q < kSymMaxRow; ++q) {
      // rows of active threads are not empty; other threads read entry 0
      const int kq = active ? (q < ne ? rb + q : rb) - beg : 0;
      sj[q] = s_ci[kq];
      su[q] = s_src[kq];
    }
  }
  const double xE = (active && !SPLIT) ? x[(size_t)G * N + i] : 0.0;
  double sE = 0.0;
  for (int a = 0; a < nb; ++a) {
    const double* __restrict__ xa = x + (size_t)a * N;
    double s = 0.0;
    if (SPLIT && a == G) {  // uniform over the workgroup
      if (active) y[(size_t)G * N + i] = sE;
      continue;
    }
    // the row's coupling operands and b of this block, loaded ahead of the
    // sum so that they are in flight with its other loads
    const size_t ro = (size_t)a * N + i;
    double c1 = 0.0, c2 = 0.0, xo = 0.0, bo = 0.0;
    if (active) {
      if (a < G) {
        if (!SPLIT) c1 = S.d_gE[ro];
        c2 = S.d_Eg[ro];
        xo = xa[i];
      } else if (a == G) {
        c1 = S.d_EI[i];
        xo = x[(size_t)(G + 1) * N + i];
      } else if (!SPLIT) {
        c1 = S.d_IE[i];
      }
      if (RESID) bo = b[ro];
    }
    if (SYM) {
      const int ul = ue - ub;  // in [nr, kSymMaxUpper nr]: every row holds its diagonal
      const double* __restrict__ uv = S.sym_v[a];
      // every load of the block at once: the segment's staging loads, the
      // row's gathers of x_a and its values outside the segment
      double r[kSymMaxUpper], xv[kSymMaxRow], mv[kSymMaxRow];
#pragma unroll
      for (int j = 0; j < kSymMaxUpper; ++j) {
        const int k = t + j * R;
        if (k < ul) r[j] = uv[ub + k];
      }
#pragma unroll
      for (int q = 0; q < kSymMaxRow; ++q) {
        if (q < ne) {
          xv[q] = xa[sj[q]];
          if (su[q] < ub || su[q] >= ue) mv[q] = uv[su[q]];
        }
      }
      __syncthreads();  // every thread is done with the previous block
#pragma unroll
      for (int j = 0; j < kSymMaxUpper; ++j) {
        const int k = t + j * R;
        if (k < ul) s_v[k] = r[j];
      }
      __syncthreads();
      // the row's sum in entry order, as below
#pragma unroll
      for (int q = 0; q < kSymMaxRow; ++q) {
        if (q < ne) {
          const int lo = su[q] - ub;
          const bool seg = (unsigned)lo < (unsigned)ul;
          const double av = seg ? s_v[seg ? lo : 0] : mv[q];
          s += av * xv[q];
        }
      }
    } else
    for (int cb = beg; cb < end; cb += CAP) {
      const int cl = min(CAP, end - cb);
      const double* __restrict__ v = S.blk[a].v + cb;
      double r[PT];
#pragma unroll
      for (int j = 0; j < PT; ++j) r[j] = v[min(t + j * R, cl - 1)];  // cl >= 1 here
      __syncthreads();  // every thread is done with the previous chunk
      if (!one_chunk)
        for (int k = t; k < cl; k += R) s_ci[k] = ci[cb + k];
#pragma unroll
      for (int j = 0; j < PT; ++j) {
        const int k = t + j * R;
        if (k < cl) s_v[k] = r[j];
      }
      __syncthreads();
      const int kb = max(rb, cb), ke = min(re, cb + cl);
      // eight entries at a time: their gathers in flight together (the sum in
      // entry order; entries past the row's end repeat its last and are not added)
      for (int k0 = kb; k0 < ke; k0 += 8) {
        int jj[8];
        double av[8], xv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int kq = min(k0 + q, ke - 1) - cb;
          jj[q] = s_ci[kq];
          av[q] = s_v[kq];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) xv[q] = xa[jj[q]];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (k0 + q < ke) s += av[q] * xv[q];
      }
    }
    if (!active) continue;
    if (a < G) {
      if (!SPLIT) s += c1 * xE;
      sE += c2 * xo;
    } else if (a == G) {
      s += sE;
      s += c1 * xo;
    } else if (!SPLIT) {
      s += c1 * xE;
    }
    y[ro] = RESID ? bo - s : s;
  }
}

// the rest of a SPLIT block matvec, once x_E is known: the E row's stencil
// sum, then + sum_g d_Eg[g] o x_g (held in y_E) + d_EI o x_I; y_g += d_gE o x_E;
// y_I += d_IE o x_E
template <bool SYM>
__global__ void __launch_bounds__(256) k_block_matvec_finish(BlockSysDev S,
                                                             const double* __restrict__ x,
                                                             double* __restrict__ y) {
  const int G = S.G, N = S.N;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double* __restrict__ xEv = x + (size_t)G * N;
  const double xE = xEv[i];
  const int* __restrict__ rp = S.blk[0].rp;
  const int* __restrict__ ci = S.blk[0].ci;
  const double* __restrict__ v = SYM ? S.sym_v[G] : S.blk[G].v;
  double s = 0.0;
  const int kb = rp[i], ke = rp[i + 1];
  for (int k0 = kb; k0 < ke; k0 += 8) {  // as in k_block_matvec_shared
    int jj[8];
    double av[8], xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kq = min(k0 + q, ke - 1);
      jj[q] = ci[kq];
      av[q] = v[SYM ? S.sym_src[kq] : kq];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) xv[q] = xEv[jj[q]];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (k0 + q < ke) s += av[q] * xv[q];
  }
  s += y[(size_t)G * N + i];
  s += S.d_EI[i] * x[(size_t)(G + 1) * N + i];
  y[(size_t)G * N + i] = s;
  for (int g = 0; g < G; ++g) {
    const size_t r = (size_t)g * N + i;
    y[r] = y[r] + S.d_gE[r] * xE;
  }
  const size_t r = (size_t)(G + 1) * N + i;
  y[r] = y[r] + S.d_IE[i] * xE;
}

constexpr int kSharedRows = 512;

// values, pattern (once when shared, or per block with csr = true: the plain
// CSR pricing of every block), x, couplings, y (and b)
// (with the half storage: its values per block, and the value positions and
// its row starts once)
double block_matvec_bytes(const BlockSysDev& S, bool resid, bool csr) {
  const double n = (double)(S.G + 2) * S.N;
  double nnz = 0;
  for (int a = 0; a < S.G + 2; ++a) nnz += S.nnz[a];
  const double pattern = (S.shared && !csr) ? 4.0 * S.nnz[0] + 4.0 * (S.N + 1)
                                            : 4.0 * nnz + 4.0 * n;
  const double values = (S.sym && !csr)
                            ? 8.0 * S.sym_nnz * (S.G + 2) + 4.0 * S.nnz[0] + 4.0 * (S.N + 1)
                            : 8.0 * nnz;
  return values + pattern + 8.0 * (2.0 * S.G + 2.0) * S.N + 8.0 * n * (resid ? 3 : 2);
}

void block_matvec(Ctx* c, const BlockSysDev& S, const double* x, const double* b, double* y) {
  if (S.shared) {
    constexpr int R = kSharedRows;
    ProfScope ps(c, KC_BLOCK_MATVEC, block_matvec_bytes(S, b != nullptr, false),
                 ksym(c, "k_block_matvec_shared",
                      {std::to_string(R), b ? "true" : "false", "false", S.sym ? "true" : "false"}),
                 block_matvec_bytes(S, b != nullptr, true));
    const dim3 grid(cdiv(S.N, R));
    if (S.sym) {
      if (b)
        hipLaunchKernelGGL((k_block_matvec_shared<R, true, false, true>), grid, dim3(R), 0,
                           c->stream, S, x, b, y);
      else
        hipLaunchKernelGGL((k_block_matvec_shared<R, false, false, true>), grid, dim3(R), 0,
                           c->stream, S, x, b, y);
    } else if (b) {
      hipLaunchKernelGGL((k_block_matvec_shared<R, true, false, false>), grid, dim3(R), 0,
                         c->stream, S, x, b, y);
    } else {
      hipLaunchKernelGGL((k_block_matvec_shared<R, false, false, false>), grid, dim3(R), 0,
                         c->stream, S, x, b, y);
    }
    MGD_CHECK_LAUNCH();
    return;
  }
  ProfScope ps(c, KC_BLOCK_MATVEC, block_matvec_bytes(S, b != nullptr, false),
               ksym(c, "k_block_matvec", {std::to_string(tpr_of(S.tpr)), b ? "true" : "false"}));
  dispatch_tpr<BlockMatvecLaunch>(S.tpr, c, S, x, b, y);
}

// the split kernel: values of every block but E, the pattern once (per block
// in the CSR pricing), x without x_E, d_Eg, y written
static void split_bytes(const BlockSysDev& S, double& stored, double& csr) {
  const double N = S.N, G = S.G;
  double nnz = 0;
  for (int a = 0; a < S.G + 2; ++a)
    if (a != S.G) nnz += S.nnz[a];
  const double vec = 8.0 * (G + 1) * N + 8.0 * G * N + 8.0 * (G + 2) * N;
  const double values =
      S.sym ? 8.0 * S.sym_nnz * (G + 1) + 4.0 * S.nnz[0] + 4.0 * (N + 1) : 8.0 * nnz;
  stored = values + 4.0 * S.nnz[0] + 4.0 * (N + 1) + vec;
  csr = 12.0 * nnz + 4.0 * (G + 1) * (N + 1) + vec;
}

void block_matvec_split(Ctx* c, const BlockSysDev& S, const double* x, double* y,
                        hipStream_t stream) {
  MGD_REQUIRE(S.shared, "split block matvec needs the shared pattern");
  constexpr int R = kSharedRows;
  double bs = 0, bc = 0;
  if (c->profiling) split_bytes(S, bs, bc);
  ProfScope ps(c, KC_BLOCK_MATVEC, bs,
               ksym(c, "k_block_matvec_shared",
                    {std::to_string(R), "false", "true", S.sym ? "true" : "false"}),
               bc, stream);
  if (S.sym)
    hipLaunchKernelGGL((k_block_matvec_shared<R, false, true, true>), dim3(cdiv(S.N, R)), dim3(R),
                       0, stream, S, x, (const double*)nullptr, y);
  else
    hipLaunchKernelGGL((k_block_matvec_shared<R, false, true, false>), dim3(cdiv(S.N, R)), dim3(R),
                       0, stream, S, x, (const double*)nullptr, y);
  MGD_CHECK_LAUNCH();
}

void block_matvec_finish(Ctx* c, const BlockSysDev& S, const double* x, double* y) {
  // A_E (values, pattern), x_E, x_I, d_EI, d_IE, d_gE, y read and written
  const double N = S.N, G = S.G;
  const double b = 12.0 * S.nnz[S.G] + 4.0 * (N + 1) + 8.0 * 4 * N + 8.0 * G * N +
                   16.0 * (G + 2) * N;
  // with the half storage: its values and the value positions instead of the values
  const double bs = S.sym ? b - 8.0 * S.nnz[S.G] + 8.0 * S.sym_nnz + 4.0 * S.nnz[S.G] : b;
  ProfScope ps(c, KC_BLOCK_MATVEC, bs,
               ksym(c, "k_block_matvec_finish", {S.sym ? "true" : "false"}), b);
  if (S.sym)
    hipLaunchKernelGGL(k_block_matvec_finish<true>, dim3(cdiv(S.N, 256)), dim3(256), 0, c->stream,
                       S, x, y);
  else
    hipLaunchKernelGGL(k_block_matvec_finish<false>, dim3(cdiv(S.N, 256)), dim3(256), 0,
                       c->stream, S, x, y);
  MGD_CHECK_LAUNCH();
}

}  // namespace mgd
