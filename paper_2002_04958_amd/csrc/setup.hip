// AMG setup kernels: strength of connection, PMIS, classical modified
// interpolation, sorted transpose, canonical-order SpGEMM, l1 diagonal and
// the dense coarsest-level inverse.
//
// Every floating-point sum here is evaluated left to right in a fixed order
// with separately rounded products and additions (no contraction into fused
// multiply-adds), so the results are reproducible bit for bit by any other
// implementation that follows the same order.
#pragma clang fp contract(off)

#include <algorithm>
#include <climits>

#include "kernels.hpp"
#include "setup.hpp"

namespace mgd {

// ---------------------------------------------------------------------------
// copies
// ---------------------------------------------------------------------------
void csr_copy_from(Ctx* c, const mgd_csr* A, Csr<double>& out) {
  out.alloc(c, A->n_rows, A->n_cols, (int)A->nnz);
  copy_d2d(c, out.rp.get(), A->row_ptr, (size_t)A->n_rows + 1);
  copy_d2d(c, out.ci.get(), A->col_idx, (size_t)A->nnz);
  copy_d2d(c, out.v.get(), A->val, (size_t)A->nnz);
}
void csr_copy(Ctx* c, const Csr<double>& A, Csr<double>& out) {
  out.alloc(c, A.n_rows, A.n_cols, A.nnz);
  copy_d2d(c, out.rp.get(), A.rp.get(), (size_t)A.n_rows + 1);
  copy_d2d(c, out.ci.get(), A.ci.get(), (size_t)A.nnz);
  copy_d2d(c, out.v.get(), A.v.get(), (size_t)A.nnz);
}

// ---------------------------------------------------------------------------
// strength of connection
// ---------------------------------------------------------------------------
__global__ void k_strength(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, double theta, double dom,
                           uint8_t* __restrict__ S, int* __restrict__ stc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e0 = rp[i], e1 = rp[i + 1];
  double m = -INFINITY, rs = 0.0, dg = 0.0;
  for (int e = e0; e < e1; ++e) {
    const double a = v[e];
    rs = rs + a;
    if (ci[e] == i)
      dg = a;
    else if (-a > m)
      m = -a;
  }
  bool empty = !(m > 0.0);
  if (dom > 0.0 && rs >= dom * dg) empty = true;
  const double thr = theta * m;
  for (int e = e0; e < e1; ++e) {
    const int j = ci[e];
    const bool s = !empty && j != i && (-v[e] >= thr);
    S[e] = s ? 1 : 0;
    if (s) atomicAdd(&stc[j], 1);
  }
}

void strength(Ctx* c, const Csr<double>& A, double theta, double dom, DBuf<uint8_t>& S,
              DBuf<int>& stc) {
  S.alloc(c, (size_t)A.nnz);
  stc.alloc(c, (size_t)A.n_rows);
  fill<int>(c, stc.get(), 0, (size_t)A.n_rows);
  if (A.n_rows == 0) return;
  hipLaunchKernelGGL(k_strength, dim3(cdiv(A.n_rows, 256)), dim3(256), 0, c->stream, A.n_rows,
                     A.rp.get(), A.ci.get(), A.v.get(), theta, dom, S.get(), stc.get());
  MGD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// PMIS
// ---------------------------------------------------------------------------
// First output of SplitMix64 for the given state (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t splitmix64_first(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_pmis_init(int n, const int* __restrict__ stc, uint64_t seed, int level,
                            uint64_t* __restrict__ key, int8_t* __restrict__ state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t h = splitmix64_first(seed ^ ((uint64_t)level << 56) ^ (uint64_t)i) >> 32;
  key[i] = ((uint64_t)stc[i] << 32) | h;
  state[i] = stc[i] == 0 ? kF : kU;
}

__global__ void k_st_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                          const uint8_t* __restrict__ S, int* __restrict__ fillpos,
                          int* __restrict__ st_ci, int cap, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (S[e]) {
      const int p = atomicAdd(&fillpos[ci[e]], 1);
      if (p >= 0 && p < cap)
        st_ci[p] = i;
      else
        atomicOr(err, 1);
    }
}

__device__ __forceinline__ bool beats(uint64_t kj, int j, uint64_t ki, int i) {
  return kj > ki || (kj == ki && j > i);
}

__global__ void k_pmis_select(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                              const uint8_t* __restrict__ S, const int* __restrict__ st_rp,
                              const int* __restrict__ st_ci, const uint64_t* __restrict__ key,
                              const int8_t* __restrict__ state, uint8_t* __restrict__ newc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] != kU) {
    newc[i] = 0;
    return;
  }
  const uint64_t ki = key[i];
  bool best = true;
  for (int e = rp[i]; e < rp[i + 1] && best; ++e) {
    if (!S[e]) continue;
    const int j = ci[e];
    if (state[j] == kU && beats(key[j], j, ki, i)) best = false;
  }
  for (int p = st_rp[i]; p < st_rp[i + 1] && best; ++p) {
    const int j = st_ci[p];
    if (state[j] == kU && beats(key[j], j, ki, i)) best = false;
  }
  newc[i] = best ? 1 : 0;
}

__global__ void k_pmis_update(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                              const uint8_t* __restrict__ S, const uint8_t* __restrict__ newc,
                              int8_t* __restrict__ state, int* __restrict__ remaining) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool und = false;
  if (i < n && state[i] == kU) {
    if (newc[i]) {
      state[i] = kC;
    } else {
      bool dep = false;
      for (int e = rp[i]; e < rp[i + 1]; ++e)
        if (S[e] && newc[ci[e]]) {
          dep = true;
          break;
        }
      if (dep)
        state[i] = kF;
      else
        und = true;
    }
  }
  const uint64_t m = __ballot(und);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(remaining, (int)__popcll(m));
}

__global__ void k_count_undecided(int n, const int8_t* __restrict__ state,
                                  int* __restrict__ remaining) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t m = __ballot(i < n && state[i] == kU);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(remaining, (int)__popcll(m));
}

// ---------------------------------------------------------------------------
// HMIS: Ruge-Stueben first pass inside tiles of consecutive rows (one
// workgroup per tile, state in LDS), then PMIS for the points it leaves open
// ---------------------------------------------------------------------------
constexpr int kMaxHmisTile = 1024;

__device__ __forceinline__ uint64_t block_max_u64(uint64_t v, uint64_t* red) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t m = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = red[w] > m ? red[w] : m;
  __syncthreads();
  return m;
}

// One workgroup (256 threads) per tile [t0, t1).  The measure of a point is
// the number of undecided tile points depending strongly on it; the point of
// largest (measure, hash, index) with a positive measure becomes C, the
// undecided tile points depending on it become F, the measures of those new F
// points' undecided tile dependencies rise by one, then the measures of the new
// C point's undecided tile dependencies drop by one.  c0[i] = 1 for the C points.
__global__ void __launch_bounds__(256) k_rs_tiles(int n, int tile, uint64_t seed, int level,
                                                  const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const uint8_t* __restrict__ S,
                                                  const int* __restrict__ st_rp,
                                                  const int* __restrict__ st_ci,
                                                  int8_t* __restrict__ c0) {
  __shared__ int lam[kMaxHmisTile];
  __shared__ int8_t st[kMaxHmisTile];
  __shared__ uint8_t newf[kMaxHmisTile];
  __shared__ uint32_t hk[kMaxHmisTile];
  __shared__ uint64_t red[4];
  const int t0 = blockIdx.x * tile, t1 = min(n, t0 + tile), nt = t1 - t0;
  for (int i = threadIdx.x; i < nt; i += 256) {
    st[i] = 0;
    newf[i] = 0;
    hk[i] = (uint32_t)(splitmix64_first(seed ^ ((uint64_t)level << 56) ^ (uint64_t)(t0 + i)) >> 32);
    int m = 0;
    for (int e = st_rp[t0 + i]; e < st_rp[t0 + i + 1]; ++e) {
      const int j = st_ci[e];
      m += (j >= t0 && j < t1) ? 1 : 0;
    }
    lam[i] = m;
  }
  __syncthreads();
  for (int step = 0; step < nt; ++step) {
    uint64_t best = 0;
    for (int i = threadIdx.x; i < nt; i += 256) {
      if (st[i] == 0 && lam[i] > 0) {
        const uint64_t k = ((uint64_t)lam[i] << 48) | ((uint64_t)hk[i] << 16) | (uint64_t)i;
        best = k > best ? k : best;
      }
    }
    best = block_max_u64(best, red);
    if (best == 0) break;  // the same value in every thread
    const int pl = (int)(best & 0xffff), pg = t0 + pl;
    if (threadIdx.x == 0) st[pl] = 1;
    __syncthreads();
    // undecided tile points depending on the new C point become F
    for (int e = st_rp[pg] + threadIdx.x; e < st_rp[pg + 1]; e += 256) {
      const int j = st_ci[e] - t0;
      if (j >= 0 && j < nt && st[j] == 0) {
        st[j] = -1;
        newf[j] = 1;
      }
    }
    __syncthreads();
    // their undecided tile dependencies gain one
    for (int e = st_rp[pg] + threadIdx.x; e < st_rp[pg + 1]; e += 256) {
      const int j = st_ci[e] - t0;
      if (j >= 0 && j < nt && newf[j]) {
        newf[j] = 0;
        for (int f = rp[t0 + j]; f < rp[t0 + j + 1]; ++f) {
          const int k = ci[f] - t0;
          if (S[f] && k >= 0 && k < nt && st[k] == 0) atomicAdd(&lam[k], 1);
        }
      }
    }
    __syncthreads();
    // the new C point's undecided tile dependencies lose one
    for (int f = rp[pg] + threadIdx.x; f < rp[pg + 1]; f += 256) {
      const int k = ci[f] - t0;
      if (S[f] && k >= 0 && k < nt && st[k] == 0) atomicAdd(&lam[k], -1);
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < nt; i += 256) c0[t0 + i] = st[i] == 1 ? 1 : 0;
}

// HMIS initial state: first-pass C points; F for points nobody depends on or
// that depend strongly on a first-pass C point; undecided otherwise
__global__ void k_hmis_init(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                            const uint8_t* __restrict__ S, const int* __restrict__ stc,
                            const int8_t* __restrict__ c0, int8_t* __restrict__ state) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (c0[i]) {
    state[i] = kC;
    return;
  }
  bool dep = stc[i] == 0;
  for (int e = rp[i]; e < rp[i + 1] && !dep; ++e)
    if (S[e] && c0[ci[e]]) dep = true;
  state[i] = dep ? kF : kU;
}

int pmis(Ctx* c, const Csr<double>& A, const DBuf<uint8_t>& S, const DBuf<int>& stc,
         uint64_t seed, int level, DBuf<int8_t>& state, int hmis_tile) {
  const int n = A.n_rows;
  state.alloc(c, (size_t)n);
  if (n == 0) return 0;
  DBuf<uint64_t> key(c, (size_t)n);
  DBuf<uint8_t> newc(c, (size_t)n);
  DBuf<int> st_rp(c, (size_t)n + 1), fillpos(c, (size_t)n), remaining(c, 1);
  const int g = cdiv(n, 256);
  hipLaunchKernelGGL(k_pmis_init, dim3(g), dim3(256), 0, c->stream, n, stc.get(), seed, level,
                     key.get(), state.get());
  MGD_CHECK_LAUNCH();
  const int nst = exclusive_scan_total(c, stc.get(), st_rp.get(), n);
  DBuf<int> st_ci(c, (size_t)std::max(nst, 1));
  copy_d2d(c, fillpos.get(), st_rp.get(), (size_t)n);
  hipLaunchKernelGGL(k_st_fill, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(),
                     S.get(), fillpos.get(), st_ci.get(), nst, c->err_flag());
  MGD_CHECK_LAUNCH();
  c->check_device_errors("transposed strength graph");
  check_index_structure(c, n, n, nst, st_rp.get(), st_ci.get(), "transposed strength graph");
  if (hmis_tile > 0) {
    DBuf<int8_t> c0(c, (size_t)n);
    hipLaunchKernelGGL(k_rs_tiles, dim3(cdiv(n, hmis_tile)), dim3(256), 0, c->stream, n, hmis_tile,
                       seed, level, A.rp.get(), A.ci.get(), S.get(), (const int*)st_rp.get(),
                       (const int*)st_ci.get(), c0.get());
    MGD_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_hmis_init, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(),
                       S.get(), stc.get(), (const int8_t*)c0.get(), state.get());
    MGD_CHECK_LAUNCH();
    c->sync();
  }
  fill<int>(c, remaining.get(), 0, 1);
  hipLaunchKernelGGL(k_count_undecided, dim3(g), dim3(256), 0, c->stream, n, state.get(),
                     remaining.get());
  MGD_CHECK_LAUNCH();
  int rounds = 0;
  while (read1(c, remaining.get()) > 0) {
    fill<int>(c, remaining.get(), 0, 1);
    hipLaunchKernelGGL(k_pmis_select, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(),
                       S.get(), st_rp.get(), st_ci.get(), key.get(), state.get(), newc.get());
    MGD_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_pmis_update, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(),
                       S.get(), newc.get(), state.get(), remaining.get());
    MGD_CHECK_LAUNCH();
    // each round decides at least the undecided row of largest (key, index)
    if (++rounds > n) fail(MGD_EHIP, "PMIS did not terminate");
  }
  return rounds;
}

// ---------------------------------------------------------------------------
// classical modified interpolation
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sgn(double x) { return (x > 0.0) - (x < 0.0); }

// position of column j in the sorted row [e0, e1), or -1
__device__ __forceinline__ int find_col(const int* __restrict__ ci, int e0, int e1, int j) {
  int lo = e0, hi = e1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (ci[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < e1 && ci[lo] == j) ? lo : -1;
}

__global__ void k_diag(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                       const double* __restrict__ v, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = find_col(ci, rp[i], rp[i + 1], i);
  d[i] = p >= 0 ? v[p] : 0.0;
}

__global__ void k_interp_count(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                               const uint8_t* __restrict__ S, const int8_t* __restrict__ st,
                               int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (st[i] == kC) {
    cnt[i] = 1;
    return;
  }
  int k = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (S[e] && st[ci[e]] == kC) ++k;
  cnt[i] = k;
}

__global__ void k_interp_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                              const double* __restrict__ v, const double* __restrict__ diag,
                              const uint8_t* __restrict__ S, const int8_t* __restrict__ st,
                              const int* __restrict__ cidx, const int* __restrict__ prp,
                              int* __restrict__ pci, double* __restrict__ pv,
                              double* __restrict__ sigma, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = prp[i];
  const int pend = prp[i + 1];
  if (st[i] == kC) {
    if (pend != p + 1) {  // the count pass gives C rows exactly one entry
      atomicOr(err, 2);
      return;
    }
    pci[p] = cidx[i];
    pv[p] = 1.0;
    return;
  }
  const int e0 = rp[i], e1 = rp[i + 1];
  // 1. sigma_ik = sum over j in C_i (ascending j) of ahat_kj, for strong F k
  for (int e = e0; e < e1; ++e) {
    const int k = ci[e];
    if (!S[e] || st[k] != kF) continue;
    const int f0 = rp[k], f1 = rp[k + 1];
    const int skk = sgn(diag[k]);
    double s = 0.0;
    int q = e0;
    for (int f = f0; f < f1; ++f) {
      const int j = ci[f];
      while (q < e1 && ci[q] < j) ++q;
      if (q < e1 && ci[q] == j && S[q] && st[j] == kC) {
        const double a = v[f];
        s = s + (sgn(a) != skk ? a : 0.0);
      }
    }
    sigma[e] = s;
  }
  // 2. modified diagonal: a_ii + weak neighbours + strong F without common C
  double at = diag[i];
  for (int e = e0; e < e1; ++e) {
    const int j = ci[e];
    if (j == i) continue;
    if (!S[e])
      at = at + v[e];
    else if (st[j] == kF && sigma[e] == 0.0)
      at = at + v[e];
  }
  // 3. weights for each strong C point, distribution over ascending k
  for (int e = e0; e < e1; ++e) {
    const int j = ci[e];
    if (!S[e] || st[j] != kC) continue;
    double num = v[e];
    for (int e2 = e0; e2 < e1; ++e2) {
      const int k = ci[e2];
      if (!S[e2] || st[k] != kF) continue;
      const double sg = sigma[e2];
      if (sg == 0.0) continue;
      const int f = find_col(ci, rp[k], rp[k + 1], j);
      if (f < 0) continue;
      const double a = v[f];
      const double ah = sgn(a) != sgn(diag[k]) ? a : 0.0;
      num = num + (v[e2] * ah) / sg;
    }
    if (p >= pend) {  // more entries than the count pass gave this row
      atomicOr(err, 1);
      return;
    }
    pci[p] = cidx[j];
    pv[p] = -num / at;
    ++p;
  }
  if (p != pend) atomicOr(err, 2);
}

__global__ void k_is_c(int n, const int8_t* __restrict__ st, int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = st[i] == kC ? 1 : 0;
}

void interpolation(Ctx* c, const Csr<double>& A, const DBuf<uint8_t>& S,
                   const DBuf<int8_t>& state, const DBuf<int>& cidx, int nc, Csr<double>& P) {
  const int n = A.n_rows;
  DBuf<int> cnt(c, (size_t)n);
  DBuf<double> diag(c, (size_t)n), sigma(c, (size_t)std::max(A.nnz, 1));
  const int g = cdiv(n, 256);
  hipLaunchKernelGGL(k_diag, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(), A.v.get(),
                     diag.get());
  MGD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_interp_count, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(),
                     S.get(), state.get(), cnt.get());
  MGD_CHECK_LAUNCH();
  P.n_rows = n;
  P.n_cols = nc;
  P.rp.alloc(c, (size_t)n + 1);
  P.nnz = exclusive_scan_total(c, cnt.get(), P.rp.get(), n);
  P.ci.alloc(c, (size_t)P.nnz);
  P.v.alloc(c, (size_t)P.nnz);
  hipLaunchKernelGGL(k_interp_fill, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(),
                     A.v.get(), diag.get(), S.get(), state.get(), cidx.get(), P.rp.get(),
                     P.ci.get(), P.v.get(), sigma.get(), c->err_flag());
  MGD_CHECK_LAUNCH();
  c->check_device_errors("interpolation fill");
}

// ---------------------------------------------------------------------------
// sorted transpose
// ---------------------------------------------------------------------------
__global__ void k_count_cols(int nnz, const int* __restrict__ ci, int* __restrict__ cnt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[ci[e]], 1);
}
__global__ void k_transpose_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                 const double* __restrict__ v, int* __restrict__ fillpos,
                                 int* __restrict__ tci, double* __restrict__ tv, int cap,
                                 int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int p = atomicAdd(&fillpos[ci[e]], 1);
    if (p < 0 || p >= cap) {
      atomicOr(err, 1);
      continue;
    }
    tci[p] = i;
    tv[p] = v[e];
  }
}
// insertion sort of each row by column (rows of a transpose are short)
__global__ void k_sort_rows(int n, const int* __restrict__ rp, int* __restrict__ ci,
                            double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e0 = rp[i], e1 = rp[i + 1];
  for (int e = e0 + 1; e < e1; ++e) {
    const int kc = ci[e];
    const double kv = v[e];
    int q = e - 1;
    while (q >= e0 && ci[q] > kc) {
      ci[q + 1] = ci[q];
      v[q + 1] = v[q];
      --q;
    }
    ci[q + 1] = kc;
    v[q + 1] = kv;
  }
}

void transpose(Ctx* c, const Csr<double>& A, Csr<double>& T) {
  T.n_rows = A.n_cols;
  T.n_cols = A.n_rows;
  T.nnz = A.nnz;
  DBuf<int> cnt(c, (size_t)std::max(A.n_cols, 1)), fillpos(c, (size_t)std::max(A.n_cols, 1));
  fill<int>(c, cnt.get(), 0, (size_t)A.n_cols);
  if (A.nnz)
    hipLaunchKernelGGL(k_count_cols, dim3(cdiv(A.nnz, 256)), dim3(256), 0, c->stream, A.nnz,
                       A.ci.get(), cnt.get());
  MGD_CHECK_LAUNCH();
  T.rp.alloc(c, (size_t)A.n_cols + 1);
  exclusive_scan(c, cnt.get(), T.rp.get(), A.n_cols);
  T.ci.alloc(c, (size_t)A.nnz);
  T.v.alloc(c, (size_t)A.nnz);
  copy_d2d(c, fillpos.get(), T.rp.get(), (size_t)A.n_cols);
  if (A.n_rows)
    hipLaunchKernelGGL(k_transpose_fill, dim3(cdiv(A.n_rows, 256)), dim3(256), 0, c->stream,
                       A.n_rows, A.rp.get(), A.ci.get(), A.v.get(), fillpos.get(), T.ci.get(),
                       T.v.get(), A.nnz, c->err_flag());
  MGD_CHECK_LAUNCH();
  c->check_device_errors("transpose");
  if (T.n_rows)
      hipLaunchKernelGGL(k_sort_rows, dim3(cdiv(T.n_rows, 256)), dim3(256), 0, c->stream, T.n_rows,
                       T.rp.get(), T.ci.get(), T.v.get());
  MGD_CHECK_LAUNCH();
  c->sync();
  check_structure(c, T, "transpose", false);
}

// ---------------------------------------------------------------------------
// SpGEMM: row-wise multiway merge.  Every output column of row i is produced
// in ascending order; its value is 0 + a_ik1 b_k1j + a_ik2 b_k2j + ... over
// the row's entries in ascending k.
// ---------------------------------------------------------------------------
template <bool FILL>
__global__ void k_spgemm(int n, const int* __restrict__ arp, const int* __restrict__ aci,
                         const double* __restrict__ av, const int* __restrict__ brp,
                         const int* __restrict__ bci, const double* __restrict__ bv,
                         int* __restrict__ head, int* __restrict__ hend,
                         const int* __restrict__ crp, int* __restrict__ cnt_or_cci,
                         double* __restrict__ cv, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e0 = arp[i], e1 = arp[i + 1];
  for (int e = e0; e < e1; ++e) {
    const int k = aci[e];
    head[e] = brp[k];
    hend[e] = brp[k + 1];
  }
  int out = FILL ? crp[i] : 0;
  const int oend = FILL ? crp[i + 1] : INT_MAX;
  for (;;) {
    int jmin = INT_MAX;
    for (int e = e0; e < e1; ++e)
      if (head[e] < hend[e]) jmin = min(jmin, bci[head[e]]);
    if (jmin == INT_MAX) break;
    double acc = 0.0;
    for (int e = e0; e < e1; ++e) {
      const int h = head[e];
      if (h < hend[e] && bci[h] == jmin) {
        if (FILL) acc = acc + av[e] * bv[h];
        head[e] = h + 1;
      }
    }
    if (FILL) {
      if (out >= oend) {  // more columns than the symbolic pass counted
        atomicOr(err, 1);
        return;
      }
      cnt_or_cci[out] = jmin;
      cv[out] = acc;
    }
    ++out;
  }
  if (!FILL) cnt_or_cci[i] = out;
  if (FILL && out != oend) atomicOr(err, 2);
}

void spgemm(Ctx* c, const Csr<double>& A, const Csr<double>& B, Csr<double>& C) {
  MGD_REQUIRE(A.n_cols == B.n_rows, "spgemm: inner dimensions differ");
  const int n = A.n_rows;
  DBuf<int> head(c, (size_t)std::max(A.nnz, 1)), hend(c, (size_t)std::max(A.nnz, 1));
  DBuf<int> cnt(c, (size_t)std::max(n, 1));
  C.n_rows = n;
  C.n_cols = B.n_cols;
  C.rp.alloc(c, (size_t)n + 1);
  const int g = cdiv(n, 128);
  if (n)
    hipLaunchKernelGGL(k_spgemm<false>, dim3(g), dim3(128), 0, c->stream, n, A.rp.get(),
                       A.ci.get(), A.v.get(), B.rp.get(), B.ci.get(), B.v.get(), head.get(),
                       hend.get(), (const int*)nullptr, cnt.get(), (double*)nullptr, c->err_flag());
  MGD_CHECK_LAUNCH();
  C.nnz = exclusive_scan_total(c, cnt.get(), C.rp.get(), n);
  C.ci.alloc(c, (size_t)C.nnz);
  C.v.alloc(c, (size_t)C.nnz);
  if (n)
    hipLaunchKernelGGL(k_spgemm<true>, dim3(g), dim3(128), 0, c->stream, n, A.rp.get(), A.ci.get(),
                       A.v.get(), B.rp.get(), B.ci.get(), B.v.get(), head.get(), hend.get(),
                       (const int*)C.rp.get(), C.ci.get(), C.v.get(), c->err_flag());
  MGD_CHECK_LAUNCH();
  c->check_device_errors("SpGEMM fill");
}

// ---------------------------------------------------------------------------
// aggressive coarsening: a second pass of the same coarsening over the first
// pass's C points, on their strength graph of distance two (j depends on i
// when j is in S_i or in S_k for some k in S_i), numbered by ascending fine
// index; hash keys of level + kAggressiveSalt.  The graph is the pattern of
// X Y minus its diagonal, X = the strong entries of the C rows and
// Y = I + S restricted to C columns.
// ---------------------------------------------------------------------------
constexpr int kAggressiveSalt = 64;

__global__ void k_d2x_count(int n, const int* __restrict__ rp, const uint8_t* __restrict__ S,
                            const int8_t* __restrict__ st, const int* __restrict__ cidx,
                            int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || st[i] != kC) return;
  int k = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) k += S[e] ? 1 : 0;
  cnt[cidx[i]] = k;
}
__global__ void k_d2x_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const uint8_t* __restrict__ S, const int8_t* __restrict__ st,
                           const int* __restrict__ cidx, const int* __restrict__ xrp,
                           int* __restrict__ xci, double* __restrict__ xv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || st[i] != kC) return;
  int p = xrp[cidx[i]];
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (S[e]) {
      xci[p] = ci[e];
      xv[p] = 1.0;
      ++p;
    }
}
__global__ void k_d2y_count(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                            const uint8_t* __restrict__ S, const int8_t* __restrict__ st,
                            int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int k = st[i] == kC ? 1 : 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) k += (S[e] && st[ci[e]] == kC) ? 1 : 0;
  cnt[i] = k;
}
// row i of Y: i itself when it is C, and its strong C dependencies, in
// ascending coarse index (strength never flags the diagonal)
__global__ void k_d2y_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const uint8_t* __restrict__ S, const int8_t* __restrict__ st,
                           const int* __restrict__ cidx, const int* __restrict__ yrp,
                           int* __restrict__ yci, double* __restrict__ yv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = yrp[i];
  bool self = st[i] == kC;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int j = ci[e];
    if (self && j > i) {
      yci[p] = cidx[i];
      yv[p] = 1.0;
      ++p;
      self = false;
    }
    if (S[e] && st[j] == kC) {
      yci[p] = cidx[j];
      yv[p] = 1.0;
      ++p;
    }
  }
  if (self) {
    yci[p] = cidx[i];
    yv[p] = 1.0;
  }
}
__global__ void k_offdiag_count(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int k = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) k += ci[e] != i ? 1 : 0;
  cnt[i] = k;
}
__global__ void k_offdiag_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                               const int* __restrict__ orp, int* __restrict__ oci,
                               double* __restrict__ ov) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = orp[i];
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] != i) {
      oci[p] = ci[e];
      ov[p] = 1.0;
      ++p;
    }
}
__global__ void k_d2_combine(int n, const int8_t* __restrict__ st1, const int* __restrict__ cidx1,
                             const int8_t* __restrict__ st2, int8_t* __restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  st[i] = (st1[i] == kC && st2[cidx1[i]] == kC) ? kC : kF;
}

// state: first-pass C/F splitting in, final splitting out; returns the rounds
// of the second pass
int aggressive_split(Ctx* c, const Csr<double>& A, const DBuf<uint8_t>& S,
                     const DBuf<int>& cidx1, int n1, uint64_t seed, int level, int hmis_tile,
                     DBuf<int8_t>& state) {
  const int n = A.n_rows;
  const int g = cdiv(n, 256);
  Csr<double> X, Y, Z, G2;
  {
    DBuf<int> cnt(c, (size_t)std::max(n1, 1));
    hipLaunchKernelGGL(k_d2x_count, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), S.get(),
                       state.get(), cidx1.get(), cnt.get());
    MGD_CHECK_LAUNCH();
    X.n_rows = n1;
    X.n_cols = n;
    X.rp.alloc(c, (size_t)n1 + 1);
    X.nnz = exclusive_scan_total(c, cnt.get(), X.rp.get(), n1);
    X.ci.alloc(c, (size_t)std::max(X.nnz, 1));
    X.v.alloc(c, (size_t)std::max(X.nnz, 1));
    hipLaunchKernelGGL(k_d2x_fill, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(),
                       S.get(), state.get(), cidx1.get(), (const int*)X.rp.get(), X.ci.get(),
                       X.v.get());
    MGD_CHECK_LAUNCH();
  }
  {
    DBuf<int> cnt(c, (size_t)n);
    hipLaunchKernelGGL(k_d2y_count, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(),
                       S.get(), state.get(), cnt.get());
    MGD_CHECK_LAUNCH();
    Y.n_rows = n;
    Y.n_cols = n1;
    Y.rp.alloc(c, (size_t)n + 1);
    Y.nnz = exclusive_scan_total(c, cnt.get(), Y.rp.get(), n);
    Y.ci.alloc(c, (size_t)std::max(Y.nnz, 1));
    Y.v.alloc(c, (size_t)std::max(Y.nnz, 1));
    hipLaunchKernelGGL(k_d2y_fill, dim3(g), dim3(256), 0, c->stream, n, A.rp.get(), A.ci.get(),
                       S.get(), state.get(), cidx1.get(), (const int*)Y.rp.get(), Y.ci.get(),
                       Y.v.get());
    MGD_CHECK_LAUNCH();
  }
  check_structure(c, X, "distance-two graph: X", false);
  check_structure(c, Y, "distance-two graph: Y", false);
  spgemm(c, X, Y, Z);
  check_structure(c, Z, "distance-two graph", false);
  {
    const int g1 = cdiv(n1, 256);
    DBuf<int> cnt(c, (size_t)std::max(n1, 1));
    hipLaunchKernelGGL(k_offdiag_count, dim3(g1), dim3(256), 0, c->stream, n1, Z.rp.get(),
                       Z.ci.get(), cnt.get());
    MGD_CHECK_LAUNCH();
    G2.n_rows = G2.n_cols = n1;
    G2.rp.alloc(c, (size_t)n1 + 1);
    G2.nnz = exclusive_scan_total(c, cnt.get(), G2.rp.get(), n1);
    G2.ci.alloc(c, (size_t)std::max(G2.nnz, 1));
    G2.v.alloc(c, (size_t)std::max(G2.nnz, 1));
    hipLaunchKernelGGL(k_offdiag_fill, dim3(g1), dim3(256), 0, c->stream, n1, Z.rp.get(),
                       Z.ci.get(), (const int*)G2.rp.get(), G2.ci.get(), G2.v.get());
    MGD_CHECK_LAUNCH();
  }
  DBuf<uint8_t> S2(c, (size_t)std::max(G2.nnz, 1));
  fill<uint8_t>(c, S2.get(), (uint8_t)1, (size_t)G2.nnz);
  DBuf<int> stc2(c, (size_t)std::max(n1, 1));
  fill<int>(c, stc2.get(), 0, (size_t)n1);
  if (G2.nnz)
    hipLaunchKernelGGL(k_count_cols, dim3(cdiv(G2.nnz, 256)), dim3(256), 0, c->stream, G2.nnz,
                       G2.ci.get(), stc2.get());
  MGD_CHECK_LAUNCH();
  DBuf<int8_t> st2;
  const int rounds = pmis(c, G2, S2, stc2, seed, level + kAggressiveSalt, st2, hmis_tile);
  DBuf<int8_t> out(c, (size_t)n);
  hipLaunchKernelGGL(k_d2_combine, dim3(g), dim3(256), 0, c->stream, n, state.get(), cidx1.get(),
                     (const int8_t*)st2.get(), out.get());
  MGD_CHECK_LAUNCH();
  c->sync();
  state = std::move(out);
  return rounds;
}

// ---------------------------------------------------------------------------
// multipass interpolation (Stueben 2001): C rows are the identity; a point of
// pass m (its nearest C point is m strong dependencies away) interpolates
// through its strong dependencies P_i of pass m - 1:
//   alpha = (sum of negative off-diagonal a_ij) / (sum_{j in P_i} a_ij),
//   d = a_ii + (sum of the other off-diagonal a_ij),
//   w_ik = -(alpha * (0 + sum_{j in P_i, ascending} a_ij w_jk)) / d.
// Rows are built pass by pass into a buffer per pass; off[i], len[i] locate
// row i in its pass's buffer.  Points no chain reaches get empty rows.
// ---------------------------------------------------------------------------
__global__ void k_mp_init(int n, const int8_t* __restrict__ st, const int* __restrict__ cidx,
                          int* __restrict__ pass, int* __restrict__ off, int* __restrict__ len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool isc = st[i] == kC;
  pass[i] = isc ? 0 : -1;
  off[i] = isc ? cidx[i] : 0;
  len[i] = isc ? 1 : 0;
}
__global__ void k_iota(int n, int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = i;
}
// pass m for every unreached point with a strong dependency of pass m - 1
// (a point set in this launch reads as m or -1, never as m - 1)
__global__ void k_mp_assign(int n, int m, const int* __restrict__ rp, const int* __restrict__ ci,
                            const uint8_t* __restrict__ S, int* __restrict__ pass,
                            int* __restrict__ added) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool hit = false;
  if (i < n && pass[i] < 0)
    for (int e = rp[i]; e < rp[i + 1]; ++e)
      if (S[e] && pass[ci[e]] == m - 1) {
        hit = true;
        break;
      }
  if (hit) pass[i] = m;
  const uint64_t b = __ballot(hit);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(added, (int)__popcll(b));
}
template <bool FILL>
__global__ void k_mp_rows(int n, int m, const int* __restrict__ rp, const int* __restrict__ ci,
                          const double* __restrict__ v, const uint8_t* __restrict__ S,
                          const int* __restrict__ pass, const int* __restrict__ bci,
                          const double* __restrict__ bv, int* __restrict__ off,
                          int* __restrict__ len, int* __restrict__ head, int* __restrict__ hend,
                          const int* __restrict__ orp, int* __restrict__ cnt_or_oci,
                          double* __restrict__ ov, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (pass[i] != m) {
    if (!FILL) cnt_or_oci[i] = 0;
    return;
  }
  const int e0 = rp[i], e1 = rp[i + 1];
  double dg = 0.0, sn = 0.0, sp = 0.0, sP = 0.0;
  for (int e = e0; e < e1; ++e) {
    const int j = ci[e];
    const double a = v[e];
    if (j == i)
      dg = a;
    else if (a < 0.0)
      sn = sn + a;
    else
      sp = sp + a;
    if (S[e] && pass[j] == m - 1) {
      sP = sP + a;
      head[e] = off[j];
      hend[e] = off[j] + len[j];
    } else {
      head[e] = 0;
      hend[e] = 0;
    }
  }
  const double alpha = sn / sP, d = dg + sp;
  int out = FILL ? orp[i] : 0;
  const int oend = FILL ? orp[i + 1] : INT_MAX;
  for (;;) {
    int kmin = INT_MAX;
    for (int e = e0; e < e1; ++e)
      if (head[e] < hend[e]) kmin = min(kmin, bci[head[e]]);
    if (kmin == INT_MAX) break;
    double acc = 0.0;
    for (int e = e0; e < e1; ++e) {
      const int h = head[e];
      if (h < hend[e] && bci[h] == kmin) {
        if (FILL) acc = acc + v[e] * bv[h];
        head[e] = h + 1;
      }
    }
    if (FILL) {
      if (out >= oend) {  // more columns than the count pass gave this row
        atomicOr(err, 1);
        return;
      }
      cnt_or_oci[out] = kmin;
      ov[out] = -(alpha * acc) / d;
    }
    ++out;
  }
  if (!FILL) {
    cnt_or_oci[i] = out;
  } else {
    if (out != oend) atomicOr(err, 2);
    off[i] = orp[i];
    len[i] = out - orp[i];
  }
}
__global__ void k_mp_copy(int n, int m, const int* __restrict__ pass, const int* __restrict__ off,
                          const int* __restrict__ len, const int* __restrict__ bci,
                          const double* __restrict__ bv, const int* __restrict__ prp,
                          int* __restrict__ pci, double* __restrict__ pv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || pass[i] != m) return;
  const int o = off[i], p = prp[i];
  for (int q = 0; q < len[i]; ++q) {
    pci[p + q] = bci[o + q];
    pv[p + q] = bv[o + q];
  }
}

void multipass_interpolation(Ctx* c, const Csr<double>& A, const DBuf<uint8_t>& S,
                             const DBuf<int8_t>& state, const DBuf<int>& cidx, int nc,
                             Csr<double>& P) {
  const int n = A.n_rows;
  const int g = cdiv(n, 256);
  DBuf<int> pass(c, (size_t)n), off(c, (size_t)n), len(c, (size_t)n), added(c, 1);
  hipLaunchKernelGGL(k_mp_init, dim3(g), dim3(256), 0, c->stream, n, state.get(), cidx.get(),
                     pass.get(), off.get(), len.get());
  MGD_CHECK_LAUNCH();
  std::vector<DBuf<int>> bci;
  std::vector<DBuf<double>> bv;
  bci.emplace_back(c, (size_t)std::max(nc, 1));
  bv.emplace_back(c, (size_t)std::max(nc, 1));
  hipLaunchKernelGGL(k_iota, dim3(cdiv(std::max(nc, 1), 256)), dim3(256), 0, c->stream, nc,
                     bci[0].get());
  MGD_CHECK_LAUNCH();
  fill<double>(c, bv[0].get(), 1.0, (size_t)nc);
  DBuf<int> head(c, (size_t)std::max(A.nnz, 1)), hend(c, (size_t)std::max(A.nnz, 1));
  DBuf<int> cnt(c, (size_t)n), orp(c, (size_t)n + 1);
  for (int m = 1;; ++m) {
    if (m > n) fail(MGD_EHIP, "multipass interpolation did not terminate");
    fill<int>(c, added.get(), 0, 1);
    hipLaunchKernelGGL(k_mp_assign, dim3(g), dim3(256), 0, c->stream, n, m, A.rp.get(),
                       A.ci.get(), S.get(), pass.get(), added.get());
    MGD_CHECK_LAUNCH();
    if (read1(c, added.get()) == 0) break;
    hipLaunchKernelGGL(k_mp_rows<false>, dim3(g), dim3(256), 0, c->stream, n, m, A.rp.get(),
                       A.ci.get(), A.v.get(), S.get(), (const int*)pass.get(),
                       (const int*)bci[m - 1].get(), (const double*)bv[m - 1].get(), off.get(),
                       len.get(), head.get(), hend.get(), (const int*)nullptr, cnt.get(),
                       (double*)nullptr, c->err_flag());
    MGD_CHECK_LAUNCH();
    const int tot = exclusive_scan_total(c, cnt.get(), orp.get(), n);
    bci.emplace_back(c, (size_t)std::max(tot, 1));
    bv.emplace_back(c, (size_t)std::max(tot, 1));
    hipLaunchKernelGGL(k_mp_rows<true>, dim3(g), dim3(256), 0, c->stream, n, m, A.rp.get(),
                       A.ci.get(), A.v.get(), S.get(), (const int*)pass.get(),
                       (const int*)bci[m - 1].get(), (const double*)bv[m - 1].get(), off.get(),
                       len.get(), head.get(), hend.get(), (const int*)orp.get(), bci[m].get(),
                       bv[m].get(), c->err_flag());
    MGD_CHECK_LAUNCH();
    c->check_device_errors("multipass interpolation");
  }
  P.n_rows = n;
  P.n_cols = nc;
  P.rp.alloc(c, (size_t)n + 1);
  P.nnz = exclusive_scan_total(c, len.get(), P.rp.get(), n);
  P.ci.alloc(c, (size_t)std::max(P.nnz, 1));
  P.v.alloc(c, (size_t)std::max(P.nnz, 1));
  for (int m = 0; m < (int)bci.size(); ++m)
    hipLaunchKernelGGL(k_mp_copy, dim3(g), dim3(256), 0, c->stream, n, m, (const int*)pass.get(),
                       (const int*)off.get(), (const int*)len.get(), (const int*)bci[m].get(),
                       (const double*)bv[m].get(), (const int*)P.rp.get(), P.ci.get(), P.v.get());
  MGD_CHECK_LAUNCH();
  c->sync();
}

// ---------------------------------------------------------------------------
// l1 diagonal
// ---------------------------------------------------------------------------
__global__ void k_l1diag(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                         const double* __restrict__ v, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e0 = rp[i], e1 = rp[i + 1];
  double acc = 0.0;
  for (int e = e0; e < e1; ++e)
    if (ci[e] == i) acc = v[e];
  for (int e = e0; e < e1; ++e)
    if (ci[e] != i) acc = acc + fabs(v[e]);
  d[i] = acc;
}
void plain_diagonal(Ctx* c, const Csr<double>& A, double* d) {
  if (!A.n_rows) return;
  hipLaunchKernelGGL(k_diag, dim3(cdiv(A.n_rows, 256)), dim3(256), 0, c->stream, A.n_rows,
                     A.rp.get(), A.ci.get(), A.v.get(), d);
  MGD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Jones-Plassmann colouring (multicolour Gauss-Seidel): every stored
// off-diagonal entry of A is an edge in both directions; in round c every
// uncoloured row whose (hash32(seed, level, i), i) beats all uncoloured
// neighbours gets colour c
// ---------------------------------------------------------------------------
__global__ void k_jp_select(int n, int round, uint64_t seed, int level,
                            const int* __restrict__ rp, const int* __restrict__ ci,
                            const int* __restrict__ trp, const int* __restrict__ tci,
                            const int* __restrict__ colour, uint8_t* __restrict__ win) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (colour[i] >= 0) {
    win[i] = 0;
    return;
  }
  const uint64_t salt = seed ^ ((uint64_t)level << 56);
  const uint32_t ki = (uint32_t)(splitmix64_first(salt ^ (uint64_t)i) >> 32);
  bool best = true;
  for (int e = rp[i]; e < rp[i + 1] && best; ++e) {
    const int j = ci[e];
    if (j == i || colour[j] >= 0) continue;
    const uint32_t kj = (uint32_t)(splitmix64_first(salt ^ (uint64_t)j) >> 32);
    if (kj > ki || (kj == ki && j > i)) best = false;
  }
  for (int e = trp[i]; e < trp[i + 1] && best; ++e) {
    const int j = tci[e];
    if (j == i || colour[j] >= 0) continue;
    const uint32_t kj = (uint32_t)(splitmix64_first(salt ^ (uint64_t)j) >> 32);
    if (kj > ki || (kj == ki && j > i)) best = false;
  }
  win[i] = best ? 1 : 0;
}
__global__ void k_jp_assign(int n, int round, const uint8_t* __restrict__ win,
                            int* __restrict__ colour, int* __restrict__ remaining) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool left = false;
  if (i < n) {
    if (win[i]) colour[i] = round;
    left = colour[i] < 0;
  }
  const uint64_t m = __ballot(left);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(remaining, (int)__popcll(m));
}

int jp_colouring(Ctx* c, const Csr<double>& A, uint64_t seed, int level, DBuf<int>& colour) {
  const int n = A.n_rows;
  colour.alloc(c, (size_t)std::max(n, 1));
  if (n == 0) return 0;
  fill<int>(c, colour.get(), -1, (size_t)n);
  Csr<double> T;
  transpose(c, A, T);
  DBuf<uint8_t> win(c, (size_t)n);
  DBuf<int> remaining(c, 1);
  const int g = cdiv(n, 256);
  int round = 0;
  for (;;) {
    fill<int>(c, remaining.get(), 0, 1);
    hipLaunchKernelGGL(k_jp_select, dim3(g), dim3(256), 0, c->stream, n, round, seed, level,
                       A.rp.get(), A.ci.get(), (const int*)T.rp.get(), (const int*)T.ci.get(),
                       (const int*)colour.get(), win.get());
    MGD_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_jp_assign, dim3(g), dim3(256), 0, c->stream, n, round,
                       (const uint8_t*)win.get(), colour.get(), remaining.get());
    MGD_CHECK_LAUNCH();
    ++round;
    if (read1(c, remaining.get()) == 0) break;
    // every round colours at least the uncoloured row of largest (key, index)
    if (round > n) fail(MGD_EHIP, "colouring did not terminate");
  }
  return round;
}

void l1_diagonal(Ctx* c, const Csr<double>& A, double* d) {
  if (!A.n_rows) return;
  hipLaunchKernelGGL(k_l1diag, dim3(cdiv(A.n_rows, 256)), dim3(256), 0, c->stream, A.n_rows,
                     A.rp.get(), A.ci.get(), A.v.get(), d);
  MGD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// dense inverse of the coarsest matrix (FP64): LU with partial pivoting
// (first row of maximum magnitude), then one triangular solve pair per
// column of the identity.  One workgroup; n <= dense_max.
// ---------------------------------------------------------------------------
__global__ void k_csr_to_dense(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                               const double* __restrict__ v, double* __restrict__ M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) M[(size_t)i * n + ci[e]] = v[e];
}

__global__ void __launch_bounds__(1024) k_lu(int n, double* __restrict__ M, int* __restrict__ piv,
                                             int* __restrict__ singular) {
  __shared__ double sval[1024];
  __shared__ int sidx[1024];
  const int t = threadIdx.x;
  for (int col = 0; col < n; ++col) {
    // pivot search: max |M[r][col]|, smallest r on ties
    double best = -1.0;
    int bi = INT_MAX;
    for (int r = col + t; r < n; r += 1024) {
      const double a = fabs(M[(size_t)r * n + col]);
      if (a > best) {
        best = a;
        bi = r;
      }
    }
    sval[t] = best;
    sidx[t] = bi;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
      if (t < s) {
        const double ov = sval[t + s];
        const int oi = sidx[t + s];
        if (ov > sval[t] || (ov == sval[t] && oi < sidx[t])) {
          sval[t] = ov;
          sidx[t] = oi;
        }
      }
      __syncthreads();
    }
    const int p = sidx[0];
    const double pv = sval[0];
    __syncthreads();
    if (!(pv > 0.0)) {
      if (t == 0) singular[0] = 1;
      return;
    }
    if (t == 0) piv[col] = p;
    if (p != col)
      for (int j = t; j < n; j += 1024) {
        const double tmp = M[(size_t)col * n + j];
        M[(size_t)col * n + j] = M[(size_t)p * n + j];
        M[(size_t)p * n + j] = tmp;
      }
    __syncthreads();
    const double d = M[(size_t)col * n + col];
    for (int r = col + 1 + t; r < n; r += 1024) M[(size_t)r * n + col] = M[(size_t)r * n + col] / d;
    __syncthreads();
    const int m = n - col - 1;
    for (long q = t; q < (long)m * m; q += 1024) {
      const int r = col + 1 + (int)(q / m);
      const int j = col + 1 + (int)(q % m);
      M[(size_t)r * n + j] = M[(size_t)r * n + j] - M[(size_t)r * n + col] * M[(size_t)col * n + j];
    }
    __syncthreads();
  }
}

// inverse column j: solve L U x = P e_j; written column-major inv[j*n + i]
__global__ void k_lu_inverse(int n, const double* __restrict__ M, const int* __restrict__ piv,
                             double* __restrict__ inv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double* x = inv + (size_t)j * n;
  for (int i = 0; i < n; ++i) x[i] = (i == j) ? 1.0 : 0.0;
  for (int i = 0; i < n; ++i) {  // apply the row interchanges in order
    const int p = piv[i];
    if (p != i) {
      const double t = x[i];
      x[i] = x[p];
      x[p] = t;
    }
  }
  for (int i = 0; i < n; ++i) {  // unit lower
    double s = x[i];
    for (int k = 0; k < i; ++k) s = s - M[(size_t)i * n + k] * x[k];
    x[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {  // upper
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s = s - M[(size_t)i * n + k] * x[k];
    x[i] = s / M[(size_t)i * n + i];
  }
}

bool dense_inverse(Ctx* c, const Csr<double>& A, DBuf<double>& inv) {
  const int n = A.n_rows;
  inv.alloc(c, (size_t)n * n);
  if (n == 0) return true;
  DBuf<double> M(c, (size_t)n * n);
  DBuf<int> piv(c, (size_t)n), sing(c, 1);
  fill<double>(c, M.get(), 0.0, (size_t)n * n);
  fill<int>(c, sing.get(), 0, 1);
  hipLaunchKernelGGL(k_csr_to_dense, dim3(cdiv(n, 256)), dim3(256), 0, c->stream, n, A.rp.get(),
                     A.ci.get(), A.v.get(), M.get());
  MGD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_lu, dim3(1), dim3(1024), 0, c->stream, n, M.get(), piv.get(), sing.get());
  MGD_CHECK_LAUNCH();
  if (read1(c, sing.get())) return false;
  hipLaunchKernelGGL(k_lu_inverse, dim3(cdiv(n, 64)), dim3(64), 0, c->stream, n,
                     (const double*)M.get(), (const int*)piv.get(), inv.get());
  MGD_CHECK_LAUNCH();
  c->sync();
  return true;
}

// ---------------------------------------------------------------------------
// hierarchy driver
// ---------------------------------------------------------------------------
void amg_build(Ctx* c, Csr<double>&& A0, const amg_params& p, SetupHierarchy& H) {
  H.levels.clear();
  Csr<double> A = std::move(A0);
  for (int lvl = 0;; ++lvl) {
    const int n = A.n_rows;
    SetupLevel L;
    if (n <= p.coarse_max || lvl == p.max_levels - 1 || lvl == MGD_MAX_LEVELS - 1) {
      L.A = std::move(A);
      H.levels.push_back(std::move(L));
      break;
    }
    const std::string at = " (level " + std::to_string(lvl) + ", " + std::to_string(n) + " rows)";
    DBuf<uint8_t> S;
    DBuf<int> stc;
    StepScope st_strength("amg setup: strength" + at);
    strength(c, A, p.strength_theta, p.dominance_theta, S, stc);
    DBuf<int8_t> state;
    StepScope st_pmis("amg setup: pmis" + at);
    int rounds = pmis(c, A, S, stc, p.seed, lvl, state, p.coarsening == 1 ? p.hmis_tile : 0);
    StepScope st_cnum("amg setup: coarse numbering" + at);
    DBuf<int> isc(c, (size_t)n), cidx(c, (size_t)n + 1);
    hipLaunchKernelGGL(k_is_c, dim3(cdiv(n, 256)), dim3(256), 0, c->stream, n, state.get(),
                       isc.get());
    MGD_CHECK_LAUNCH();
    int nc = exclusive_scan_total(c, isc.get(), cidx.get(), n);
    const bool aggressive = lvl < p.aggressive_levels;
    if (aggressive && nc > 0) {
      StepScope st_agg("amg setup: aggressive second pass" + at);
      rounds += aggressive_split(c, A, S, cidx, nc, p.seed, lvl,
                                 p.coarsening == 1 ? p.hmis_tile : 0, state);
      hipLaunchKernelGGL(k_is_c, dim3(cdiv(n, 256)), dim3(256), 0, c->stream, n, state.get(),
                         isc.get());
      MGD_CHECK_LAUNCH();
      nc = exclusive_scan_total(c, isc.get(), cidx.get(), n);
    }
    if (nc == 0 || 10LL * nc > 9LL * n) {  // stalled coarsening: this is the coarsest level
      L.A = std::move(A);
      H.levels.push_back(std::move(L));
      break;
    }
    Csr<double> P, R, AP, Ac;
    {
      StepScope st("amg setup: interpolation" + at);
      if (aggressive)
        multipass_interpolation(c, A, S, state, cidx, nc, P);
      else
        interpolation(c, A, S, state, cidx, nc, P);
      check_structure(c, P, "interpolation", false);
    }
    {
      StepScope st("amg setup: transpose of P" + at);
      transpose(c, P, R);
    }
    {
      StepScope st("amg setup: A P" + at);
      spgemm(c, A, P, AP);
      check_structure(c, AP, "A P", false);
    }
    {
      StepScope st("amg setup: R (A P)" + at);
      spgemm(c, R, AP, Ac);
      check_structure(c, Ac, "coarse operator", true);
    }
    L.A = std::move(A);
    L.cf = std::move(state);
    L.P = std::move(P);
    L.nc = nc;
    L.pmis_rounds = rounds;
    H.levels.push_back(std::move(L));
    A = std::move(Ac);
  }
  if (p.smoother == 1) {
    for (size_t l = 0; l < H.levels.size(); ++l) {
      StepScope st("amg setup: colouring (level " + std::to_string(l) + ")");
      auto& L = H.levels[l];
      L.ncolours = jp_colouring(c, L.A, p.seed, (int)l, L.colour);
    }
  }
  SetupLevel& last = H.levels.back();
  if (last.A.n_rows <= p.dense_max) {
    StepScope st("amg setup: coarsest LU (" + std::to_string(last.A.n_rows) + " rows)");
    H.coarse_kind = 0;
    if (!dense_inverse(c, last.A, H.coarse_inv))
      fail(MGD_ESINGULAR, "zero pivot in the coarsest-level LU");
  } else {
    H.coarse_kind = 1;
  }
}

}  // namespace mgd
