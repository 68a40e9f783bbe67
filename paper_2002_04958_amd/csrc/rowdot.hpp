// Row dot products for CSR kernels: a row is handled by a group of TPR
// consecutive lanes of one wavefront (TPR = 1 .. 64), which stride over the
// row's entries and combine with butterfly shuffles inside the group.
#pragma once
#include <hip/hip_runtime.h>

namespace mgd {

template <int TPR, typename AT, typename MT, typename XT>
__device__ __forceinline__ AT row_dot(const int* __restrict__ rp, const int* __restrict__ ci,
                                      const MT* __restrict__ v, const XT* __restrict__ x, int row,
                                      int lane) {
  AT s = 0;
  const int e1 = rp[row + 1];
  // eight of the lane's entries at a time, their gathers in flight together
  // (loads past the row's end masked off); the lane's sum stays in entry order
  for (int e = rp[row] + lane; e < e1; e += 8 * TPR) {
    int j[8];
    AT a[8], xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (e + q * TPR < e1) {
        j[q] = ci[e + q * TPR];
        a[q] = (AT)v[e + q * TPR];
      }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (e + q * TPR < e1) xv[q] = (AT)x[j[q]];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (e + q * TPR < e1) s += a[q] * xv[q];
  }
  if (TPR > 1) {
#pragma unroll
    for (int off = TPR / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, TPR);
  }
  return s;
}

// Dispatch a functor templated on TPR for runtime tpr in {1,2,4,...,64}.
template <template <int> class K, typename... Args>
inline void dispatch_tpr(int tpr, Args&&... args) {
  switch (tpr) {
    case 1: K<1>::run(args...); break;
    case 2: K<2>::run(args...); break;
    case 4: K<4>::run(args...); break;
    case 8: K<8>::run(args...); break;
    case 16: K<16>::run(args...); break;
    case 32: K<32>::run(args...); break;
    default: K<64>::run(args...); break;
  }
}

// The group width dispatch_tpr actually launches for a requested width.
inline int tpr_of(int tpr) {
  return (tpr == 1 || tpr == 2 || tpr == 4 || tpr == 8 || tpr == 16 || tpr == 32) ? tpr : 64;
}

// Group width for an average row length (used when no tuned value exists).
inline int default_tpr(double avg_row) {
  if (avg_row <= 12) return 1;
  if (avg_row <= 24) return 2;
  if (avg_row <= 48) return 4;
  if (avg_row <= 96) return 8;
  if (avg_row <= 192) return 16;
  return 32;
}

}  // namespace mgd
