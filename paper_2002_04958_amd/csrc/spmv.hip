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

double block_matvec_bytes(const BlockSysDev& S, bool resid) {
  const double n = (double)(S.G + 2) * S.N;
  double nnz = 0;
  for (int a = 0; a < S.G + 2; ++a) nnz += S.nnz[a];
  return 12.0 * nnz + 4.0 * n + 8.0 * (2.0 * S.G + 2.0) * S.N + 8.0 * n * (resid ? 3 : 2);
}

void block_matvec(Ctx* c, const BlockSysDev& S, const double* x, const double* b, double* y) {
  ProfScope ps(c, KC_BLOCK_MATVEC, block_matvec_bytes(S, b != nullptr),
               ksym(c, "k_block_matvec", {std::to_string(tpr_of(S.tpr)), b ? "true" : "false"}));
  dispatch_tpr<BlockMatvecLaunch>(S.tpr, c, S, x, b, y);
}

}  // namespace mgd
