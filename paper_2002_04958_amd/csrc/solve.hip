// Solve-phase structures and kernels: union construction, CF-l1-Jacobi
// half-sweeps, residual, restriction, prolongation, dense coarsest solve,
// and the V(n_pre, n_post) cycle driver.
#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>

#include "kernels.hpp"
#include "rowdot.hpp"
#include "solve.hpp"

namespace mgd {

// ===========================================================================
// union construction
// ===========================================================================
// The kernels below take a C/F marker only where one exists (members with a
// coarser level); members without one are all-F and use the _allf variants.
// Per-row choices are written as arithmetic on both candidates rather than as
// a select between kernel arguments under a divergent branch.
__global__ void k_flags(int n, const int8_t* __restrict__ cf, int* __restrict__ isc,
                        int* __restrict__ isf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cf[i] == kC ? 1 : 0;
  isc[i] = c;
  isf[i] = 1 - c;
}

// stored index of every member row (C rows from cbase, F rows from fbase);
// perm[stored] = off + natural
__global__ void k_map_rows(int n, const int8_t* __restrict__ cf, const int* __restrict__ cidx,
                           const int* __restrict__ fidx, int cbase, int fbase, int off,
                           int* __restrict__ srow, int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cf[i] == kC ? 1 : 0;
  const int sc = cbase + cidx[i], sf = fbase + fidx[i];
  const int s = sf + c * (sc - sf);
  srow[i] = s;
  perm[s] = off + i;
}
__global__ void k_map_rows_allf(int n, int fbase, int off, int* __restrict__ srow,
                                int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  srow[i] = fbase + i;
  perm[fbase + i] = off + i;
}

// every stored row must be hit exactly once before the map drives any write
__global__ void k_count_hits(int n, const int* __restrict__ srow, int nS, int* __restrict__ hits,
                             int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = srow[i];
  if (s < 0 || s >= nS) {
    atomicOr(bad, 1);
    return;
  }
  atomicAdd(&hits[s], 1);
}
__global__ void k_check_hits(int nS, const int* __restrict__ hits, int* __restrict__ bad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nS && hits[s] != 1) atomicOr(bad, 2);
}

// row lengths into the stored order: all rows, or F rows only (W)
__global__ void k_row_len(int n, const int* __restrict__ rp, const int* __restrict__ srow,
                          int* __restrict__ len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  len[srow[i]] = rp[i + 1] - rp[i];
}
__global__ void k_row_len_f(int n, const int* __restrict__ rp, const int* __restrict__ srow,
                            int sbase, const int8_t* __restrict__ cf, int* __restrict__ len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (cf[i] == kC) return;
  len[srow[i] - sbase] = rp[i + 1] - rp[i];
}

// copy rows into the stored order (columns shifted by coloff): all rows, or F rows only
__device__ __forceinline__ void copy_row(const int* __restrict__ rp, const int* __restrict__ ci,
                                         const double* __restrict__ v, int i, int coloff, int p,
                                         int pend, int* __restrict__ dci, double* __restrict__ dv,
                                         int* __restrict__ err) {
  if (rp[i + 1] - rp[i] != pend - p) {  // target row length differs from the source row
    atomicOr(err, 4);
    return;
  }
  for (int e = rp[i]; e < rp[i + 1]; ++e, ++p) {
    dci[p] = ci[e] + coloff;
    dv[p] = v[e];
  }
}
__global__ void k_row_copy(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, const int* __restrict__ srow, int coloff,
                           const int* __restrict__ drp, int* __restrict__ dci,
                           double* __restrict__ dv, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = srow[i];
  copy_row(rp, ci, v, i, coloff, drp[s], drp[s + 1], dci, dv, err);
}
__global__ void k_row_copy_f(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                             const double* __restrict__ v, const int* __restrict__ srow, int sbase,
                             const int8_t* __restrict__ cf, int coloff,
                             const int* __restrict__ drp, int* __restrict__ dci,
                             double* __restrict__ dv, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (cf[i] == kC) return;
  const int s = srow[i] - sbase;
  copy_row(rp, ci, v, i, coloff, drp[s], drp[s + 1], dci, dv, err);
}

__global__ void k_iota(int n, int first, int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = first + i;
}
// inverse of a permutation given as perm[k] (k < n), with a range check
template <typename T>
__global__ void k_dinv_nat(int n, int nC, const int* __restrict__ iperm,
                           const T* __restrict__ dinv, T* __restrict__ dn) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int k = iperm[p];
  dn[p] = k < nC ? dinv[k] : (T)0;
}
__global__ void k_invert(int n, const int* __restrict__ perm, int* __restrict__ inv,
                         int* __restrict__ err) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = perm[k];
  if (i < 0 || i >= n) {
    atomicOr(err, 8);
    return;
  }
  inv[i] = k;
}
// columns through a map (entry order kept)
__global__ void k_remap(long long nnz, const int* __restrict__ map, int ncols_map,
                        int* __restrict__ ci, int* __restrict__ err) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int j = ci[e];
  if (j < 0 || j >= ncols_map) {
    atomicOr(err, 16);
    return;
  }
  ci[e] = map[j];
}
// row gather: out row k = in row src[k]
__global__ void k_gather_len(int n, const int* __restrict__ rp, const int* __restrict__ src,
                             int* __restrict__ len) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) len[k] = rp[src[k] + 1] - rp[src[k]];
}
__global__ void k_gather_rows(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                              const double* __restrict__ v, const int* __restrict__ src,
                              const int* __restrict__ orp, int* __restrict__ oci,
                              double* __restrict__ ov, int* __restrict__ err) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = src[k];
  int p = orp[k];
  if (orp[k + 1] - p != rp[i + 1] - rp[i]) {
    atomicOr(err, 32);
    return;
  }
  for (int e = rp[i]; e < rp[i + 1]; ++e, ++p) {
    oci[p] = ci[e];
    ov[p] = v[e];
  }
}
// out[idx[i]] = v[i]
__global__ void k_scatter_int(int n, const int* __restrict__ idx, const int* __restrict__ v,
                              int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[idx[i]] = v[i];
}

// out[i] = a[b[i]] with b[i] in [0, na)
__global__ void k_compose(int n, const int* __restrict__ a, int na, const int* __restrict__ bidx,
                          int* __restrict__ out, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = bidx[i];
  if (j < 0 || j >= na) {
    atomicOr(err, 64);
    return;
  }
  out[i] = a[j];
}

template <typename T>
__global__ void k_dinv(int n, const double* __restrict__ d, const int* __restrict__ srow,
                       T* __restrict__ dinv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dinv[srow[i]] = (T)(1.0 / d[i]);
}

struct MemberAtLevel {
  const SetupHierarchy* H;
  const SetupLevel* lev;
  int kind;  // 0 coarsening, 1 relaxed last level, 2 dense last level
  int off, n, nc;
};

// Level products of the construction pass, before the stored-order finalisation.
template <typename T>
struct BuildLevel {
  int n = 0, nS = 0, nC = 0, n_coarse = 0;
  Csr<double> A;   // nS rows (stored order), natural columns
  Csr<double> W;   // nS - nC rows, coarse natural columns
  Csr<double> Wt;  // n_coarse rows (coarse natural), F-index columns
  DBuf<int> perm;  // stored -> natural (nS)
  DBuf<int> cnat;  // C-block position -> coarse natural index (nC); empty: identity
  DBuf<T> dinv;    // nS
  DBuf<T> dgs;     // 1 / a_ii (multicolour Gauss-Seidel)
  std::vector<std::array<int, 4>> cranges;  // per colour: C-block [lo, hi), F-block [lo, hi)
  long long nnz_C = 0;
  struct Dense {
    int off, n;
    const double* inv;
  };
  std::vector<Dense> dense;  // natural offsets
};
template <typename T>
static void finalize_levels(Ctx* c, std::vector<BuildLevel<T>>& bl, Union<T>& U, int autotune);

// Host-side verification of a union level (MGD_DEBUG_UNION=1): the stored-row
// map is a permutation, row lengths and row pointers agree with the members'
// matrices, and every copied row equals its source row.  Throws with the first
// mismatch; used to diagnose, never needed for correct operation.
static bool debug_union() {
  static const bool on = [] {
    const char* e = std::getenv("MGD_DEBUG_UNION");
    return e && e[0] == '1';
  }();
  return on;
}
static void verify_flags_and_scans(Ctx* c, int n, const int8_t* cf_d, const int* isc_d,
                                   const int* isf_d, const int* cidx_d, const int* fidx_d) {
  std::vector<int8_t> cf(n, 0);
  std::vector<int> isc(n), isf(n), cidx((size_t)n + 1), fidx((size_t)n + 1);
  if (cf_d) copy_d2h(c, cf.data(), cf_d, (size_t)n);
  copy_d2h(c, isc.data(), isc_d, (size_t)n);
  copy_d2h(c, isf.data(), isf_d, (size_t)n);
  copy_d2h(c, cidx.data(), cidx_d, (size_t)n + 1);
  copy_d2h(c, fidx.data(), fidx_d, (size_t)n + 1);
  int sc = 0, sf = 0;
  for (int i = 0; i <= n; ++i) {
    if (cidx[i] != sc || fidx[i] != sf) {
      std::string ctx = "";
      for (int k = std::max(0, i - 3); k < std::min(n, i + 4); ++k)
        ctx += " [" + std::to_string(k) + ": cf " + std::to_string((int)cf[k]) + " isc " +
               std::to_string(isc[k]) + " isf " + std::to_string(isf[k]) + " cidx " +
               std::to_string(cidx[k]) + " fidx " + std::to_string(fidx[k]) + "]";
      fail(MGD_EHIP, "union debug: scan mismatch at " + std::to_string(i) + " of " +
                         std::to_string(n) + ": cidx " + std::to_string(cidx[i]) + " expected " +
                         std::to_string(sc) + ", fidx " + std::to_string(fidx[i]) + " expected " +
                         std::to_string(sf) + ";" + ctx);
    }
    if (i == n) break;
    const int want = cf_d && cf[i] == kC ? 1 : 0;
    if (isc[i] != want || isf[i] != 1 - want)
      fail(MGD_EHIP, "union debug: flags at " + std::to_string(i) + ": cf " +
                         std::to_string((int)cf[i]) + " isc " + std::to_string(isc[i]) + " isf " +
                         std::to_string(isf[i]));
    sc += isc[i];
    sf += isf[i];
  }
}
static void verify_union_level(Ctx* c, const std::vector<MemberAtLevel>& ms,
                               const std::vector<DBuf<int>>& srows, int nS, const int* alen_d,
                               const Csr<double>* Ad) {
  std::vector<int> alen(nS), seen(nS, -1);
  copy_d2h(c, alen.data(), alen_d, (size_t)nS);
  std::vector<int> arp, aci;
  if (Ad) {
    arp.resize((size_t)nS + 1);
    aci.resize((size_t)std::max(Ad->nnz, 1));
    copy_d2h(c, arp.data(), Ad->rp.get(), (size_t)nS + 1);
    copy_d2h(c, aci.data(), Ad->ci.get(), (size_t)Ad->nnz);
    long long acc = 0;
    for (int s = 0; s < nS; ++s) {
      if (arp[s] != acc)
        fail(MGD_EHIP, "union debug: row_ptr[" + std::to_string(s) + "] = " +
                           std::to_string(arp[s]) + ", scan of lengths gives " + std::to_string(acc));
      acc += alen[s];
    }
    if (arp[nS] != acc || acc != Ad->nnz)
      fail(MGD_EHIP, "union debug: row_ptr[nS] = " + std::to_string(arp[nS]) + ", total " +
                         std::to_string(acc) + ", nnz " + std::to_string(Ad->nnz));
  }
  for (size_t q = 0; q < ms.size(); ++q) {
    const auto& m = ms[q];
    if (m.kind == 2) continue;
    const int n = m.n;
    std::vector<int> srow(n), rp((size_t)n + 1), ci((size_t)std::max(m.lev->A.nnz, 1));
    copy_d2h(c, srow.data(), srows[q].get(), (size_t)n);
    copy_d2h(c, rp.data(), m.lev->A.rp.get(), (size_t)n + 1);
    copy_d2h(c, ci.data(), m.lev->A.ci.get(), (size_t)m.lev->A.nnz);
    for (int i = 0; i < n; ++i) {
      const int s = srow[i];
      const std::string at = "member " + std::to_string(q) + " row " + std::to_string(i) +
                             " -> stored " + std::to_string(s);
      if (s < 0 || s >= nS) fail(MGD_EHIP, "union debug: " + at + " out of range");
      if (seen[s] >= 0)
        fail(MGD_EHIP, "union debug: " + at + " also taken by row " + std::to_string(seen[s]));
      seen[s] = i;
      const int len = rp[i + 1] - rp[i];
      if (alen[s] != len)
        fail(MGD_EHIP, "union debug: " + at + " length " + std::to_string(alen[s]) + ", source " +
                           std::to_string(len));
      if (Ad)
        for (int k = 0; k < len; ++k)
          if (aci[(size_t)arp[s] + k] != ci[(size_t)rp[i] + k] + m.off)
            fail(MGD_EHIP, "union debug: " + at + " entry " + std::to_string(k) + " column " +
                               std::to_string(aci[(size_t)arp[s] + k]) + ", source " +
                               std::to_string(ci[(size_t)rp[i] + k]) + " + " + std::to_string(m.off));
    }
  }
}

constexpr int kSortWindow = 128;  // two 64-row slices: less padding, gathers stay local

template <typename T>
std::unique_ptr<Union<T>> build_union(Ctx* c, const std::vector<const SetupHierarchy*>& members,
                                      int n_pre, int n_post, int autotune, int smoother) {
  auto U = std::make_unique<Union<T>>();
  U->n_pre = n_pre;
  U->n_post = n_post;
  U->gs = smoother == 1;
  U->members = (int)members.size();
  std::vector<BuildLevel<T>> built;
  size_t maxL = 0;
  for (auto* H : members) maxL = std::max(maxL, H->levels.size());
  for (size_t l = 0; l < maxL; ++l) {
    StepScope st("solve-phase build: level " + std::to_string(l) + " of " +
                 std::to_string(members.size()) + " hierarchies");
    std::vector<MemberAtLevel> ms;
    int off = 0, nCtot = 0, nFtot = 0, ncoarse = 0;
    for (auto* H : members) {
      if (l >= H->levels.size()) continue;
      MemberAtLevel m;
      m.H = H;
      m.lev = &H->levels[l];
      const bool last = (l + 1 == H->levels.size());
      m.kind = !last ? 0 : (H->coarse_kind == 1 ? 1 : 2);
      m.off = off;
      m.n = m.lev->A.n_rows;
      m.nc = m.kind == 0 ? m.lev->nc : 0;
      off += m.n;
      if (m.kind == 0) {
        nCtot += m.nc;
        nFtot += m.n - m.nc;
        ncoarse += m.nc;
      } else if (m.kind == 1) {
        nFtot += m.n;
      }
      ms.push_back(m);
    }
    BuildLevel<T> lv;
    lv.n = off;
    lv.nC = nCtot;
    lv.nS = nCtot + nFtot;
    lv.n_coarse = ncoarse;
    const int nS = lv.nS, nF = nFtot;
    lv.perm.alloc(c, (size_t)std::max(nS, 1));
    lv.dinv.alloc(c, (size_t)std::max(nS, 1));
    if (smoother == 1) lv.dgs.alloc(c, (size_t)std::max(nS, 1));
    DBuf<int> alen(c, (size_t)nS + 1), wlen(c, (size_t)nF + 1), hits(c, (size_t)nS + 1);
    fill<int>(c, alen.get(), 0, (size_t)nS + 1);
    fill<int>(c, wlen.get(), 0, (size_t)nF + 1);
    fill<int>(c, hits.get(), 0, (size_t)nS + 1);
    int* bad = c->err_flag();
    std::vector<DBuf<int>> srows;
    int cbase = 0, fbase = nCtot;
    long long want_a = 0, want_w = 0;  // nnz the stored matrix and W must end with
    for (auto& m : ms) {
      DBuf<int> srow;
      if (m.kind == 2) {
        srows.push_back(std::move(srow));
        continue;
      }
      const int n = m.n, g = cdiv(n, 256);
      srow.alloc(c, (size_t)n);
      const int8_t* cf = m.kind == 0 ? m.lev->cf.get() : nullptr;
      if (m.kind == 0) {
        DBuf<int> isc(c, n), isf(c, n), cidx(c, (size_t)n + 1), fidx(c, (size_t)n + 1);
        hipLaunchKernelGGL(k_flags, dim3(g), dim3(256), 0, c->stream, n, cf, isc.get(), isf.get());
        MGD_CHECK_LAUNCH();
        exclusive_scan(c, isc.get(), cidx.get(), n);
        exclusive_scan(c, isf.get(), fidx.get(), n);
        if (debug_union()) verify_flags_and_scans(c, n, cf, isc.get(), isf.get(), cidx.get(), fidx.get());
        hipLaunchKernelGGL(k_map_rows, dim3(g), dim3(256), 0, c->stream, n, cf,
                           (const int*)cidx.get(), (const int*)fidx.get(), cbase, fbase, m.off,
                           srow.get(), lv.perm.get());
        MGD_CHECK_LAUNCH();
        c->sync();
      } else {
        hipLaunchKernelGGL(k_map_rows_allf, dim3(g), dim3(256), 0, c->stream, n, fbase, m.off,
                           srow.get(), lv.perm.get());
        MGD_CHECK_LAUNCH();
      }
      hipLaunchKernelGGL(k_count_hits, dim3(g), dim3(256), 0, c->stream, n,
                         (const int*)srow.get(), nS, hits.get(), bad);
      MGD_CHECK_LAUNCH();
      want_a += m.lev->A.nnz;
      if (m.kind == 0) want_w += (long long)m.lev->P.nnz - m.nc;
      cbase += m.nc;
      fbase += (m.kind == 0) ? m.n - m.nc : m.n;
      srows.push_back(std::move(srow));
    }
    if (nS > 0) {
      hipLaunchKernelGGL(k_check_hits, dim3(cdiv(nS, 256)), dim3(256), 0, c->stream, nS,
                         (const int*)hits.get(), bad);
      MGD_CHECK_LAUNCH();
    }
    c->check_device_errors("stored-row map of a solve-phase level");
    // Below the finest level, rows of the C-block and of the F-block are ordered
    // by decreasing length (stable) within windows of kSortWindow rows, so that
    // 64-row slices hold rows of similar length while neighbouring rows stay
    // close; the coarse numbering stays member order and is kept in cnat.
    // With multicolour Gauss-Seidel the blocks are ordered by colour instead, so
    // each colour is one range of the C-block and one of the F-block.
    if (nS > 0 && (smoother == 1 || l > 0)) {
      for (size_t q = 0; q < ms.size(); ++q) {
        const auto& m = ms[q];
        if (m.kind == 2) continue;
        if (smoother == 1) {
          MGD_REQUIRE(m.lev->colour.p, "internal: level without colours");
          hipLaunchKernelGGL(k_scatter_int, dim3(cdiv(m.n, 256)), dim3(256), 0, c->stream, m.n,
                             (const int*)srows[q].get(), (const int*)m.lev->colour.get(),
                             alen.get());
        } else {
          hipLaunchKernelGGL(k_row_len, dim3(cdiv(m.n, 256)), dim3(256), 0, c->stream, m.n,
                             m.lev->A.rp.get(), (const int*)srows[q].get(), alen.get());
        }
        MGD_CHECK_LAUNCH();
      }
      std::vector<int> len(nS), pm(nS), qpos(nS), cn(std::max(nCtot, 1));
      copy_d2h(c, len.data(), alen.get(), (size_t)nS);
      copy_d2h(c, pm.data(), lv.perm.get(), (size_t)nS);
      std::vector<int> order(nS);
      for (int k = 0; k < nS; ++k) order[k] = k;
      if (smoother == 1) {  // ascending colour (len holds colours here)
        auto by_col = [&](int a, int b2) { return len[a] < len[b2]; };
        std::stable_sort(order.begin(), order.begin() + nCtot, by_col);
        std::stable_sort(order.begin() + nCtot, order.end(), by_col);
        int ncol = 0;
        for (int k = 0; k < nS; ++k) ncol = std::max(ncol, len[k] + 1);
        lv.cranges.assign(ncol, {0, 0, 0, 0});
        for (int cc = 0; cc < ncol; ++cc) lv.cranges[cc] = {nCtot, nCtot, nS, nS};
        for (int k = nS - 1; k >= 0; --k) {  // first and last position of each colour
          const int cc = len[order[k]], blk = k < nCtot ? 0 : 2;
          lv.cranges[cc][blk] = k;
        }
        for (int k = 0; k < nS; ++k) {
          const int cc = len[order[k]], blk = k < nCtot ? 1 : 3;
          lv.cranges[cc][blk] = k + 1;
        }
        for (auto& r : lv.cranges) {  // colours absent from a block: empty range
          if (r[1] <= r[0]) r[0] = r[1] = 0;
          if (r[3] <= r[2]) r[2] = r[3] = 0;
        }
      } else {
        // windows of kSortWindow rows keep neighbouring rows close together
        auto by_len = [&](int a, int b2) { return len[a] > len[b2]; };
        for (int w0 = 0; w0 < nCtot; w0 += kSortWindow)
          std::stable_sort(order.begin() + w0, order.begin() + std::min(nCtot, w0 + kSortWindow),
                           by_len);
        for (int w0 = nCtot; w0 < nS; w0 += kSortWindow)
          std::stable_sort(order.begin() + w0, order.begin() + std::min(nS, w0 + kSortWindow),
                           by_len);
      }
      std::vector<int> pm2(nS);
      for (int k = 0; k < nS; ++k) {
        qpos[order[k]] = k;  // old position -> new position
        pm2[k] = pm[order[k]];
      }
      for (int k = 0; k < nCtot; ++k) cn[k] = order[k];  // coarse index of C position k
      DBuf<int> qd(c, (size_t)nS);
      copy_h2d(c, qd.get(), qpos.data(), (size_t)nS);
      copy_h2d(c, lv.perm.get(), pm2.data(), (size_t)nS);
      lv.cnat.alloc(c, (size_t)std::max(nCtot, 1));
      copy_h2d(c, lv.cnat.get(), cn.data(), (size_t)std::max(nCtot, 1));
      for (size_t q = 0; q < ms.size(); ++q) {
        if (ms[q].kind == 2) continue;
        hipLaunchKernelGGL(k_remap, dim3(cdiv(ms[q].n, 256)), dim3(256), 0, c->stream,
                           (long long)ms[q].n, (const int*)qd.get(), nS, srows[q].get(), bad);
        MGD_CHECK_LAUNCH();
      }
      fill<int>(c, alen.get(), 0, (size_t)nS + 1);
      c->check_device_errors("length order of a solve-phase level");
    }
    // the map is a permutation: lengths, diagonals
    for (size_t q = 0; q < ms.size(); ++q) {
      auto& m = ms[q];
      if (m.kind == 2) continue;
      const int n = m.n, g = cdiv(n, 256);
      hipLaunchKernelGGL(k_row_len, dim3(g), dim3(256), 0, c->stream, n, m.lev->A.rp.get(),
                         (const int*)srows[q].get(), alen.get());
      MGD_CHECK_LAUNCH();
      if (m.kind == 0)
        hipLaunchKernelGGL(k_row_len_f, dim3(g), dim3(256), 0, c->stream, n, m.lev->P.rp.get(),
                           (const int*)srows[q].get(), nCtot, (const int8_t*)m.lev->cf.get(),
                           wlen.get());
      MGD_CHECK_LAUNCH();
      DBuf<double> d(c, (size_t)n);
      l1_diagonal(c, m.lev->A, d.get());
      hipLaunchKernelGGL(k_dinv<T>, dim3(g), dim3(256), 0, c->stream, n, (const double*)d.get(),
                         (const int*)srows[q].get(), lv.dinv.get());
      MGD_CHECK_LAUNCH();
      if (smoother == 1) {
        plain_diagonal(c, m.lev->A, d.get());
        hipLaunchKernelGGL(k_dinv<T>, dim3(g), dim3(256), 0, c->stream, n, (const double*)d.get(),
                           (const int*)srows[q].get(), lv.dgs.get());
        MGD_CHECK_LAUNCH();
      }
      c->sync();
    }
    if (debug_union()) verify_union_level(c, ms, srows, nS, alen.get(), nullptr);
    // stored matrix (natural columns)
    Csr<double> Ad, Wd, Wtd;
    Ad.n_rows = nS;
    Ad.n_cols = lv.n;
    Ad.rp.alloc(c, (size_t)nS + 1);
    Ad.nnz = exclusive_scan_total(c, alen.get(), Ad.rp.get(), nS);
    if (Ad.nnz != want_a)
      fail(MGD_EHIP, "internal check failed: stored level matrix has " + std::to_string(Ad.nnz) +
                         " entries, its members " + std::to_string(want_a) + step_suffix());
    Ad.ci.alloc(c, (size_t)std::max(Ad.nnz, 1));
    Ad.v.alloc(c, (size_t)std::max(Ad.nnz, 1));
    Wd.n_rows = nF;
    Wd.n_cols = ncoarse;
    Wd.rp.alloc(c, (size_t)nF + 1);
    Wd.nnz = exclusive_scan_total(c, wlen.get(), Wd.rp.get(), nF);
    if (Wd.nnz != want_w)
      fail(MGD_EHIP, "internal check failed: W has " + std::to_string(Wd.nnz) + " entries, " +
                         std::to_string(want_w) + " expected" + step_suffix());
    Wd.ci.alloc(c, (size_t)std::max(Wd.nnz, 1));
    Wd.v.alloc(c, (size_t)std::max(Wd.nnz, 1));
    int coarse_off = 0;
    for (size_t q = 0; q < ms.size(); ++q) {
      auto& m = ms[q];
      if (m.kind == 2) {
        lv.dense.push_back({m.off, m.n, m.H->coarse_inv.get()});
        continue;
      }
      const int n = m.n, g = cdiv(n, 256);
      hipLaunchKernelGGL(k_row_copy, dim3(g), dim3(256), 0, c->stream, n, m.lev->A.rp.get(),
                         m.lev->A.ci.get(), m.lev->A.v.get(), (const int*)srows[q].get(), m.off,
                         (const int*)Ad.rp.get(), Ad.ci.get(), Ad.v.get(), bad);
      MGD_CHECK_LAUNCH();
      if (m.kind == 0) {
        hipLaunchKernelGGL(k_row_copy_f, dim3(g), dim3(256), 0, c->stream, n, m.lev->P.rp.get(),
                           m.lev->P.ci.get(), m.lev->P.v.get(), (const int*)srows[q].get(), nCtot,
                           (const int8_t*)m.lev->cf.get(), coarse_off, (const int*)Wd.rp.get(),
                           Wd.ci.get(), Wd.v.get(), bad);
        MGD_CHECK_LAUNCH();
        coarse_off += m.nc;
      }
    }
    c->check_device_errors("row copy into a solve-phase level");
    if (debug_union()) verify_union_level(c, ms, srows, nS, alen.get(), &Ad);
    check_structure(c, Ad, "union level matrix", false);
    check_structure(c, Wd, "union interpolation", false);
    if (ncoarse > 0) transpose(c, Wd, Wtd);
    if (nS > 0) lv.nnz_C = read1(c, Ad.rp.get() + nCtot);
    lv.A = std::move(Ad);
    lv.W = std::move(Wd);
    lv.Wt = std::move(Wtd);
    built.push_back(std::move(lv));
    if (ncoarse == 0) break;
  }
  finalize_levels(c, built, *U, autotune);
  {
    // level 0 seen from the natural side, for entry kernels that read their
    // inputs in natural order: the inverse permutation and d^-1 of C rows
    ULevel<T>& l0 = U->L[0];
    const int nX = l0.nX, g = cdiv(std::max(nX, 1), 256);
    l0.iperm.alloc(c, (size_t)std::max(nX, 1));
    l0.dinv_nat.alloc(c, (size_t)std::max(nX, 1));
    if (nX > 0) {
      hipLaunchKernelGGL(k_invert, dim3(g), dim3(256), 0, c->stream, nX,
                         (const int*)l0.perm.get(), l0.iperm.get(), c->err_flag());
      MGD_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_dinv_nat<T>, dim3(g), dim3(256), 0, c->stream, nX, l0.nC,
                         (const int*)l0.iperm.get(), (const T*)l0.dinv.get(), l0.dinv_nat.get());
      MGD_CHECK_LAUNCH();
    }
    c->check_device_errors("natural-order map of level 0");
  }
  U->build_tail(c);
  c->sync();
  return U;
}

// ===========================================================================
// solve kernels (stored order)
// ===========================================================================
// Iterate gathers.  A level's iterate has a C region [0, nC) and an F region
// [nC, nS) that alternate independently between two buffers, and a dense
// region [nS, nX) kept in the first buffer.  The region is chosen by index
// arithmetic on a buffer distance (a select of values, never a branch).
template <typename T>
struct GatherCF {
  const T* base;        // buffer holding the C region
  ptrdiff_t f_minus_c;  // (buffer holding the F region) - base, in elements
  int nC;
  __device__ __forceinline__ T operator()(int j) const {
    return base[j + (j < nC ? 0 : f_minus_c)];
  }
};
template <typename T>
struct GatherCFD {
  const T* base;  // C region buffer
  ptrdiff_t f_minus_c, d_minus_c;
  int nC, nS;
  __device__ __forceinline__ T operator()(int j) const {
    const ptrdiff_t o = j < nC ? 0 : (j < nS ? f_minus_c : d_minus_c);
    return base[j + o];
  }
};
template <typename T>
struct Gather1 {
  const T* x;
  __device__ __forceinline__ T operator()(int j) const { return x[j]; }
};
template <typename T>
struct GatherPerm {  // natural vector seen in stored order
  const T* x;
  const int* perm;
  __device__ __forceinline__ T operator()(int j) const { return x[perm[j]]; }
};
template <typename T>
struct GatherCOnly {  // first F half-sweep: F values are still zero
  const T* xc;
  int nC;
};

// position of row `row` in its slice: o its first value, oc its first column
// code, w the slice width; for SELL16 the slice's two column bases (fb < 0:
// the slice keeps 32-bit columns, oc then counts 32-bit words)
template <int FMT>
__device__ __forceinline__ void sell_slice(const int* __restrict__ rp, int row, int& o, int& oc,
                                           int& w, int& cb, int& fb) {
  if (FMT == kFmtSELL16) {
    const int s4 = 4 * (row >> 6);
    o = rp[s4] + (row & 63);
    w = (rp[s4 + 4] - rp[s4]) >> 6;
    cb = rp[s4 + 2];
    fb = rp[s4 + 3];
    oc = (fb < 0 ? rp[s4 + 1] >> 1 : rp[s4 + 1]) + (row & 63);
  } else {
    o = rp[row >> 6] + (row & 63);
    oc = o;
    w = (rp[(row >> 6) + 1] - rp[row >> 6]) >> 6;
    cb = fb = 0;
  }
}
__device__ __forceinline__ int sell16_decode(unsigned u, int cb, int fb) {
  return (u & 0x8000u) ? fb + (int)(u & 0x7fffu) : cb + (int)u;
}
// column of code idx of a sliced layout: a 16-bit code (NARROW) or a 32-bit column
template <bool NARROW>
__device__ __forceinline__ int sell_col(const int* __restrict__ ci, int idx, int cb, int fb) {
  if (NARROW) return sell16_decode(reinterpret_cast<const uint16_t*>(ci)[idx], cb, fb);
  return ci[idx];
}
// sum of a_rj g(j) over one sliced row (values from o, column codes from oc)
template <bool NARROW, typename T, typename G>
__device__ __forceinline__ T sell_row(const int* __restrict__ ci, const T* __restrict__ v,
                                      const G& g, int o, int oc, int w, int cb, int fb) {
  T s = 0;
  int e = 0;
  for (; e + 4 <= w; e += 4) {  // four entries' loads in flight (sum order unchanged)
    int j[4];
    T a[4], x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) j[q] = sell_col<NARROW>(ci, oc + 64 * (e + q), cb, fb);
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = v[o + 64 * (e + q)];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = g(j[q]);
#pragma unroll
    for (int q = 0; q < 4; ++q) s += a[q] * x[q];
  }
  for (; e < w; ++e) s += v[o + 64 * e] * g(sell_col<NARROW>(ci, oc + 64 * e, cb, fb));
  return s;
}
// the same over the C columns only (j < nC), F columns weighted zero
template <bool NARROW, typename T>
__device__ __forceinline__ T sell_row_c(const int* __restrict__ ci, const T* __restrict__ v,
                                        const T* __restrict__ xc, int nC, int o, int oc, int w,
                                        int cb, int fb) {
  T s = 0;
  int e = 0;
  for (; e + 4 <= w; e += 4) {
    int j[4];
    T a[4], x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) j[q] = sell_col<NARROW>(ci, oc + 64 * (e + q), cb, fb);
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = j[q] < nC ? v[o + 64 * (e + q)] : (T)0;
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = xc[j[q] < nC ? j[q] : 0];
#pragma unroll
    for (int q = 0; q < 4; ++q) s += a[q] * x[q];
  }
  for (; e < w; ++e) {
    const int j = sell_col<NARROW>(ci, oc + 64 * e, cb, fb);
    if (j < nC) s += v[o + 64 * e] * xc[j];
  }
  return s;
}

// The same sums for a wave whose 64 lanes are the 64 rows of one slice (the
// launch is aligned to slices): the slice header is read once into scalar
// registers, and the entries go in groups of eight with every column code and
// value of a group in flight together, then every gather of the group.  The
// entries past the row width in the last group load the last entry again and
// are not added, so the sum, its order and its rounding are those above.
template <bool NARROW, typename T, typename G>
__device__ __forceinline__ T sell_row8(const int* __restrict__ ci, const T* __restrict__ v,
                                       const G& g, int o, int oc, int w, int cb, int fb) {
  T s = 0;
  for (int e = 0; e < w; e += 8) {
    int j[8];
    T a[8], x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int eq = min(e + q, w - 1);
      j[q] = sell_col<NARROW>(ci, oc + 64 * eq, cb, fb);
      a[q] = v[o + 64 * eq];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = g(j[q]);
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (e + q < w) s += a[q] * x[q];
  }
  return s;
}
// C columns only: an F column's product is zero (adding a zero product leaves
// the sum as it is: a sum that starts at +0 is never -0)
template <bool NARROW, typename T>
__device__ __forceinline__ T sell_row8_c(const int* __restrict__ ci, const T* __restrict__ v,
                                         const T* __restrict__ xc, int nC, int o, int oc, int w,
                                         int cb, int fb) {
  T s = 0;
  for (int e = 0; e < w; e += 8) {
    int j[8];
    T a[8], x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int eq = min(e + q, w - 1);
      j[q] = sell_col<NARROW>(ci, oc + 64 * eq, cb, fb);
      a[q] = v[o + 64 * eq];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = xc[j[q] < nC ? j[q] : 0];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (e + q < w && j[q] < nC) s += a[q] * x[q];
  }
  return s;
}
// slice header of the wave's slice (uniform), then the lane's row in it
template <int FMT>
__device__ __forceinline__ void sell_slice_wave(const int* __restrict__ rp, int row, int& o,
                                                int& oc, int& w, int& cb, int& fb) {
  const int r64 = __builtin_amdgcn_readfirstlane(row & ~63);
  sell_slice<FMT>(rp, r64, o, oc, w, cb, fb);
  o += row & 63;
  oc += row & 63;
}

// sum over row `row` of a_rj g(j), entries in stored order; SELL uses one
// lane per row, CSR `TPR` lanes of a wavefront per row (butterfly combine).
// WAVE: sliced rows of a launch aligned to slices (every lane of a wave in the
// same slice)
template <int FMT, int TPR, bool WAVE = false, typename T, typename G>
__device__ __forceinline__ T mrow(const int* __restrict__ rp, const int* __restrict__ ci,
                                  const T* __restrict__ v, const G& g, int row, int lane) {
  T s = 0;
  if ((FMT == kFmtSELL || FMT == kFmtSELL16) && WAVE) {
    int o, oc, w, cb, fb;
    sell_slice_wave<FMT>(rp, row, o, oc, w, cb, fb);
    if (FMT == kFmtSELL16 && fb >= 0)
      s = sell_row8<true>(ci, v, g, o, oc, w, cb, fb);
    else
      s = sell_row8<false>(ci, v, g, o, oc, w, cb, fb);
  } else if (FMT == kFmtSELL || FMT == kFmtSELL16) {
    int o, oc, w, cb, fb;
    sell_slice<FMT>(rp, row, o, oc, w, cb, fb);
    // a slice is 16-bit or 32-bit as a whole: lanes diverge only in the waves
    // that straddle two slices
    if (FMT == kFmtSELL16 && fb >= 0)
      s = sell_row<true>(ci, v, g, o, oc, w, cb, fb);
    else
      s = sell_row<false>(ci, v, g, o, oc, w, cb, fb);
  } else {
    // eight of the lane's entries at a time, every column, value and gather
    // of the batch in flight together (loads past the row's end masked off),
    // the lane's sum in entry order
    const int e1 = rp[row + 1];
    for (int e = rp[row] + lane; e < e1; e += 8 * TPR) {
      int j[8];
      T a[8], x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (e + q * TPR < e1) {
          j[q] = ci[e + q * TPR];
          a[q] = v[e + q * TPR];
        }
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (e + q * TPR < e1) x[q] = g(j[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (e + q * TPR < e1) s += a[q] * x[q];
    }
    if (TPR > 1) {
#pragma unroll
      for (int off = TPR / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, TPR);
    }
  }
  return s;
}
// the same, with only C columns (the F part of the iterate is zero): F columns
// read the first C value with weight zero, so every lane issues the same loads
template <int FMT, int TPR, bool WAVE = false, typename T>
__device__ __forceinline__ T mrow_c(const int* __restrict__ rp, const int* __restrict__ ci,
                                    const T* __restrict__ v, const T* __restrict__ xc, int nC,
                                    int row, int lane) {
  T s = 0;
  if (nC == 0) return s;
  if ((FMT == kFmtSELL || FMT == kFmtSELL16) && WAVE) {
    int o, oc, w, cb, fb;
    sell_slice_wave<FMT>(rp, row, o, oc, w, cb, fb);
    if (FMT == kFmtSELL16 && fb >= 0)
      s = sell_row8_c<true>(ci, v, xc, nC, o, oc, w, cb, fb);
    else
      s = sell_row8_c<false>(ci, v, xc, nC, o, oc, w, cb, fb);
  } else if (FMT == kFmtSELL || FMT == kFmtSELL16) {
    int o, oc, w, cb, fb;
    sell_slice<FMT>(rp, row, o, oc, w, cb, fb);
    if (FMT == kFmtSELL16 && fb >= 0)
      s = sell_row_c<true>(ci, v, xc, nC, o, oc, w, cb, fb);
    else
      s = sell_row_c<false>(ci, v, xc, nC, o, oc, w, cb, fb);
  } else {
    const int e1 = rp[row + 1];
    for (int e = rp[row] + lane; e < e1; e += 8 * TPR) {  // batches as in mrow
      int j[8];
      T a[8], x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (e + q * TPR < e1) {
          j[q] = ci[e + q * TPR];
          a[q] = v[e + q * TPR];
        }
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (e + q * TPR < e1 && j[q] < nC) x[q] = xc[j[q]];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (e + q * TPR < e1 && j[q] < nC) s += a[q] * x[q];
    }
    if (TPR > 1) {
#pragma unroll
      for (int off = TPR / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, TPR);
    }
  }
  return s;
}

// Row ranges per workgroup.  Workgroups are dispatched to the device's
// chiplets (XCDs, each with its own L2) in turn; with c_xcd_rows set,
// workgroup b takes the rows of workgroup xcd_block(b), so that each chiplet
// works on one contiguous share of the rows and finds the iterate values its
// rows gather (mostly near its own rows) in its own L2.
__constant__ int c_xcd_rows = 0;
template <int FMT>
constexpr bool kSliced = FMT == kFmtSELL || FMT == kFmtSELL16;
template <int FMT>
__host__ __device__ __forceinline__ int launch_start(int r0) {
  return kSliced<FMT> ? (r0 & ~63) : r0;
}
constexpr int kXcds = 8;
__device__ __forceinline__ long xcd_block(long b, long nb) {
  const long q = nb / kXcds, r = nb % kXcds, x = b % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}
void set_xcd_rows(int on) {
  MGD_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_xcd_rows), &on, sizeof(int)));
}
// Sliced layouts (one lane per row) start at r0 rounded down to a 64-row
// slice, so that every wave works on one slice (kSliced, launch_start).
#define MGD_ROWS_TPR                                                              \
  const long b_ = c_xcd_rows ? xcd_block(blockIdx.x, gridDim.x) : (long)blockIdx.x; \
  const long t_ = b_ * blockDim.x + threadIdx.x;                                  \
  const int lane = (int)(t_ % TPR);                                               \
  const int k = launch_start<FMT>(r0) + (int)(t_ / TPR);                          \
  if (k >= r1 || k < r0) return;

// level-0 entry: B[k] = b[perm[k]]; C values of the first sweep X_C = B_C / d_C
template <typename T, bool PRE>
__global__ void k_entry(int nX, int nC, const int* __restrict__ perm, const T* __restrict__ dinv,
                        const T* __restrict__ b, T* __restrict__ B, T* __restrict__ XC) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nX) return;
  const T bb = b[perm[k]];
  B[k] = bb;
  if (k < nC) XC[k] = PRE ? bb * dinv[k] : (T)0;
}
// level-0 entry with the members' right-hand sides formed here from a block
// vector, read in natural order (member m = blockIdx.y, row i, coalesced):
// (T)(r[seg_m N + i] - coef_m[i] w[i]) written at its stored position iperm[.]
template <typename T, bool PRE>
__global__ void k_entry_nat(int N, int nC, const int* __restrict__ iperm,
                            const T* __restrict__ dinv_nat, const SegIn* __restrict__ tab,
                            const double* __restrict__ r, const T* __restrict__ w,
                            T* __restrict__ B, T* __restrict__ XC) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const SegIn d = tab[blockIdx.y];
  const size_t p = (size_t)blockIdx.y * N + i;
  double v = r[(size_t)d.seg * N + i];
  if (d.coef) v = v - d.coef[i] * (double)w[i];
  const T bb = (T)v;
  const int k = iperm[p];
  B[k] = bb;
  if (k < nC) XC[k] = PRE ? bb * dinv_nat[p] : (T)0;
}
// later cycles: B = (b - A z) in stored order (dense rows: 0), X_C as above
template <typename T, int FMT, int TPR, bool PRE>
__global__ void __launch_bounds__(256) k_entry_resid(int r0, int r1, int nS, int nC,
                                                     const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const T* __restrict__ v,
                                                     const int* __restrict__ perm,
                                                     const T* __restrict__ dinv,
                                                     const T* __restrict__ b,
                                                     const T* __restrict__ z, T* __restrict__ B,
                                                     T* __restrict__ XC) {
  MGD_ROWS_TPR
  if (k >= nS) {
    if (lane == 0) B[k] = (T)0;
    return;
  }
  const T bk = b[perm[k]];
  const T s = mrow<FMT, TPR, true>(rp, ci, v, GatherPerm<T>{z, perm}, k, lane);
  if (lane == 0) {
    const T bb = bk - s;
    B[k] = bb;
    if (k < nC) XC[k] = PRE ? bb * dinv[k] : (T)0;
  }
}

// first F half-sweep of a cycle (F iterate zero): X_F = (B_F - A_FC X_C) / d_F
template <typename T, int FMT, int TPR>
__global__ void __launch_bounds__(256) k_fhalf0(int r0, int r1, int nC, const int* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const T* __restrict__ v,
                                                const T* __restrict__ dinv,
                                                const T* __restrict__ B, const T* __restrict__ XC,
                                                T* __restrict__ Xout) {
  MGD_ROWS_TPR
  const T bk = B[k], dk = dinv[k];
  const T s = mrow_c<FMT, TPR, true>(rp, ci, v, XC, nC, k, lane);
  if (lane == 0) Xout[k] = (T)0 + (bk - s) * dk;
}

// half-sweep on rows [r0, r1): Xout = Xold + (B - A X) / d
template <typename T, int FMT, int TPR>
__global__ void __launch_bounds__(256) k_half(int r0, int r1, const int* __restrict__ rp,
                                              const int* __restrict__ ci, const T* __restrict__ v,
                                              const T* __restrict__ dinv, const T* __restrict__ B,
                                              GatherCF<T> X, const T* __restrict__ Xold,
                                              T* __restrict__ Xout) {
  MGD_ROWS_TPR
  const T xk = Xold[k], bk = B[k], dk = dinv[k];
  const T s = mrow<FMT, TPR, true>(rp, ci, v, X, k, lane);
  if (lane == 0) Xout[k] = xk + (bk - s) * dk;
}

// level-0 final C half-sweep fused with the output: z[perm[k]] = new X_C on
// C rows, the current F and dense values on the other rows
template <typename T, int FMT, int TPR>
__global__ void __launch_bounds__(256) k_half_out(int r0, int r1, int nC, int nS,
                                                  const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ v,
                                                  const T* __restrict__ dinv,
                                                  const T* __restrict__ B, GatherCF<T> X,
                                                  const T* __restrict__ XD,
                                                  const int* __restrict__ perm, T* __restrict__ z) {
  MGD_ROWS_TPR
  if (k < nC) {
    const T xk = X.base[k], bk = B[k], dk = dinv[k];
    const int pk = perm[k];
    const T s = mrow<FMT, TPR, true>(rp, ci, v, X, k, lane);
    if (lane == 0) z[pk] = xk + (bk - s) * dk;
  } else if (lane == 0) {
    if (k < nS)
      z[perm[k]] = X.base[k + X.f_minus_c];
    else
      z[perm[k]] = XD[k];
  }
}
// multicolour Gauss-Seidel on the rows of one colour, [r0, r0+n1) u [r2, r2+n2),
// in place: no two rows of a colour are coupled
template <typename T, int FMT, int TPR>
__global__ void __launch_bounds__(256) k_gs(int r0, int n1, int r2, int n2,
                                            const int* __restrict__ rp,
                                            const int* __restrict__ ci, const T* __restrict__ v,
                                            const T* __restrict__ dg, const T* __restrict__ B,
                                            T* __restrict__ X) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int lane = (int)(t % TPR);
  const int q = (int)(t / TPR);
  if (q >= n1 + n2) return;
  const int k = q < n1 ? r0 + q : r2 + (q - n1);
  const T s = mrow<FMT, TPR>(rp, ci, v, Gather1<T>{X}, k, lane);
  if (lane == 0) X[k] = X[k] + (B[k] - s) * dg[k];
}

// level-0 output without post-smoothing
template <typename T>
__global__ void k_out(int nX, GatherCFD<T> X, const int* __restrict__ perm, T* __restrict__ z) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nX) z[perm[k]] = X(k);
}

template <typename T, int FMT, int TPR>
__global__ void __launch_bounds__(256) k_resid(int r0, int r1, const int* __restrict__ rp,
                                               const int* __restrict__ ci,
                                               const T* __restrict__ v, const T* __restrict__ B,
                                               GatherCF<T> X, T* __restrict__ R) {
  MGD_ROWS_TPR
  const T bk = B[k];
  const T s = mrow<FMT, TPR, true>(rp, ci, v, X, k, lane);
  if (lane == 0) R[k] = bk - s;
}

// restriction into level l+1 (rows in its extended order):
// Bn[k] = R[cpos[k]] + sum_f Wt[k, f] R[nC + f], and its first-sweep C values
template <typename T, int FMT, int TPR, bool PRE>
__global__ void __launch_bounds__(256) k_restrict(int r0, int r1, int nC, int nCn,
                                                  const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ v,
                                                  const int* __restrict__ cpos,
                                                  const T* __restrict__ R,
                                                  const T* __restrict__ dinv_n,
                                                  T* __restrict__ Bn, T* __restrict__ XCn) {
  MGD_ROWS_TPR
  const T rc = R[cpos[k]];
  const T s = mrow<FMT, TPR, true>(rp, ci, v, Gather1<T>{R + nC}, k, lane);
  if (lane == 0) {
    const T bb = rc + s;
    Bn[k] = bb;
    if (k < nCn) XCn[k] = PRE ? bb * dinv_n[k] : (T)0;
  }
}

// prolongation: X_C[k] += E(cmap[k]) (k < nC); X_F[k] += W[k - nC, :] E
template <typename T, int FMT, int TPR>
__global__ void __launch_bounds__(256) k_prolong(int r0, int r1, int nC,
                                                 const int* __restrict__ rp,
                                                 const int* __restrict__ ci,
                                                 const T* __restrict__ v,
                                                 const int* __restrict__ cmap, GatherCFD<T> E,
                                                 T* __restrict__ XC, T* __restrict__ XF) {
  MGD_ROWS_TPR
  if (k < nC) {
    if (lane == 0) XC[k] += E(cmap[k]);
  } else {
    const T xk = XF[k];
    const T s = mrow<FMT, TPR>(rp, ci, v, E, k - nC, lane);
    if (lane == 0) XF[k] = xk + s;
  }
}

// x = A^{-1} b for every dense-solved member (FP64 arithmetic).  A workgroup
// of four waves takes 64 rows of one member; wave q sums the columns of its
// quarter in ascending order, eight column loads in flight per step, and the
// four partial sums are added in wave order.
template <typename T>
__global__ void __launch_bounds__(256) k_dense(const DenseDev* __restrict__ tab,
                                               const T* __restrict__ b, T* __restrict__ X) {
  __shared__ double part[4][64];
  const DenseDev d = tab[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // the wave: a scalar
  const int i = blockIdx.x * 64 + lane;
  const int quarter = (d.n + 3) / 4;
  const int j0 = min(d.n, q * quarter), j1 = min(d.n, j0 + quarter);
  double s = 0.0;
  if (i < d.n) {
    const double* __restrict__ col = d.inv + i;
    const T* __restrict__ bb = b + d.off;
    // eight columns at a time, the last batch cut at j1 (a scalar, like j0:
    // the branches are uniform); the sum in column order
    for (int j = j0; j < j1; j += 8) {
      double a[8], x[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (j + k < j1) {
          a[k] = col[(size_t)(j + k) * d.n];
          x[k] = (double)bb[j + k];
        }
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (j + k < j1) s += a[k] * x[k];
    }
  }
  part[q][lane] = s;
  __syncthreads();
  if (q == 0 && i < d.n)
    X[d.off + i] = (T)(((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
}

template <typename T>
__global__ void k_axpy_t(int n, const T* __restrict__ x, T* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

// ---------------------------------------------------------------------------
// persistent tail: every level from a threshold down (and back up) in one
// launch.  Each phase does what the per-level kernel of the same name does,
// with the same arithmetic, over a grid-stride loop; phases are separated by
// a grid-wide barrier.  The grid is sized so that all its workgroups are
// resident at once; a barrier wait that exceeds its spin bound reports
// through the error flag and lets the workgroup go on, so the kernel always
// ends.  The last workgroup to finish resets the counters for the next launch.
// Pointers to vectors that earlier phases write are read without __restrict__,
// so every such load goes through the memory system after the barrier's fence.
// ---------------------------------------------------------------------------
constexpr int kTailThreads = 256;
constexpr unsigned kTailSpinLimit = 1u << 17;  // about 0.1 s of polling
constexpr int kTailSyncStride = 32;  // counters 128 bytes apart
constexpr int kErrTailBarrier = 64;

__device__ __forceinline__ void tail_barrier(unsigned* arrive, unsigned target, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      // once any wait has timed out, later waits of the launch end at once
      if (++spins > kTailSpinLimit ||
          (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTailBarrier)) {
        atomicOr(err, kErrTailBarrier);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

template <int FMT, int TPR, typename T>
__device__ __forceinline__ void tail_rows(const TailOp<T>& op) {
  const long long n = (long long)(op.r1 - op.r0) * TPR;
  const long long stride = (long long)gridDim.x * kTailThreads;
  for (long long t = blockIdx.x * (long long)kTailThreads + threadIdx.x; t < n; t += stride) {
    // a group of TPR lanes shares a row: the whole group is in or out of range
    const int lane = (int)(t % TPR);
    const int k = op.r0 + (int)(t / TPR);
    if (op.kind == kTopFHalf0) {
      const T s = mrow_c<FMT, TPR>(op.rp, op.ci, op.v, op.xc, op.nC, k, lane);
      if (lane == 0) op.out[k] = (T)0 + (op.B[k] - s) * op.dinv[k];
    } else if (op.kind == kTopHalf) {
      const T s = mrow<FMT, TPR>(op.rp, op.ci, op.v, GatherCF<T>{op.xc, op.f_minus_c, op.nC}, k,
                                 lane);
      if (lane == 0) op.out[k] = op.xold[k] + (op.B[k] - s) * op.dinv[k];
    } else if (op.kind == kTopResid) {
      const T s = mrow<FMT, TPR>(op.rp, op.ci, op.v, GatherCF<T>{op.xc, op.f_minus_c, op.nC}, k,
                                 lane);
      if (lane == 0) op.out[k] = op.B[k] - s;
    } else if (op.kind == kTopRestrict) {
      const T s = mrow<FMT, TPR>(op.rp, op.ci, op.v, Gather1<T>{op.B + op.nC}, k, lane);
      if (lane == 0) {
        const T bb = op.B[op.map[k]] + s;
        op.out[k] = bb;
        if (k < op.nCn) op.out2[k] = op.pre ? bb * op.dinv[k] : (T)0;
      }
    } else {  // kTopProlong
      const GatherCFD<T> E{op.xc, (ptrdiff_t)op.f_minus_c, (ptrdiff_t)op.d_minus_c, op.nC, op.nS};
      if (k < op.nCn) {
        if (lane == 0) op.out2[k] += E(op.map[k]);
      } else {
        const T s = mrow<FMT, TPR>(op.rp, op.ci, op.v, E, k - op.nCn, lane);
        if (lane == 0) op.out[k] += s;
      }
    }
  }
}

// k_dense over virtual workgroups (member, 64-row chunk)
template <typename T>
__device__ __forceinline__ void tail_dense(const TailOp<T>& op) {
  __shared__ double part[4][64];
  const int nvb = op.ndense * op.dchunks;
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
    const DenseDev d = op.dense[vb / op.dchunks];
    const int i = (vb % op.dchunks) * 64 + lane;
    const int quarter = (d.n + 3) / 4;
    const int j0 = min(d.n, q * quarter), j1 = min(d.n, j0 + quarter);
    double sum = 0.0;
    if (i < d.n) {
      const double* __restrict__ col = d.inv + i;
      const T* bb = op.B + d.off;
      int j = j0;
      for (; j + 8 <= j1; j += 8) {
        double a[8], x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          a[k] = col[(size_t)(j + k) * d.n];
          x[k] = (double)bb[j + k];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += a[k] * x[k];
      }
      for (; j < j1; ++j) sum += col[(size_t)j * d.n] * (double)bb[j];
    }
    part[q][lane] = sum;
    __syncthreads();
    if (q == 0 && i < d.n)
      op.out[d.off + i] = (T)(((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
    __syncthreads();
  }
}

template <typename T>
__device__ __forceinline__ void tail_phase(const TailOp<T>& op) {
  if (op.kind == kTopDense) {
    tail_dense(op);
    return;
  }
  if (op.fmt == kFmtSELL) return tail_rows<kFmtSELL, 1>(op);
  if (op.fmt == kFmtSELL16) return tail_rows<kFmtSELL16, 1>(op);
  switch (op.tpr) {
    case 1: tail_rows<kFmtCSR, 1>(op); break;
    case 2: tail_rows<kFmtCSR, 2>(op); break;
    case 4: tail_rows<kFmtCSR, 4>(op); break;
    case 8: tail_rows<kFmtCSR, 8>(op); break;
    case 16: tail_rows<kFmtCSR, 16>(op); break;
    case 32: tail_rows<kFmtCSR, 32>(op); break;
    default: tail_rows<kFmtCSR, 64>(op); break;
  }
}

template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_tail(const TailOp<T>* __restrict__ ops, int nops,
                                                       unsigned* sync, int* err) {
  for (int p = 0; p < nops; ++p) {
    if (p > 0) tail_barrier(sync, (unsigned)p * gridDim.x, err);
    const TailOp<T> op = ops[p];
    tail_phase(op);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // every workgroup has passed every barrier once it counts itself out here;
    // only the counters are touched (atomically), so no data fence is needed
    const unsigned k =
        __hip_atomic_fetch_add(sync + kTailSyncStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k == gridDim.x - 1) {
      __hip_atomic_store(sync, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(sync + kTailSyncStride, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers: one row per lane (SELL) or TPR lanes per row (CSR)
// ---------------------------------------------------------------------------
template <typename T>
struct MatArgs {
  const LMat<T>* m;
};
static inline dim3 rows_grid(int rows, int tpr, int bs) { return dim3(cdiv((long long)rows * tpr, bs)); }

// Calls F.template go<FMT, TPR>() for the matrix's layout.
template <typename F>
static void with_layout(int fmt, int tpr, F&& f) {
  if (fmt == kFmtSELL) {
    f.template go<kFmtSELL, 1>();
    return;
  }
  if (fmt == kFmtSELL16) {
    f.template go<kFmtSELL16, 1>();
    return;
  }
  switch (tpr) {
    case 1: f.template go<kFmtCSR, 1>(); break;
    case 2: f.template go<kFmtCSR, 2>(); break;
    case 4: f.template go<kFmtCSR, 4>(); break;
    case 8: f.template go<kFmtCSR, 8>(); break;
    case 16: f.template go<kFmtCSR, 16>(); break;
    case 32: f.template go<kFmtCSR, 32>(); break;
    default: f.template go<kFmtCSR, 64>(); break;
  }
}
// Level and union size of the launches being profiled, appended to the kernel
// symbol as "@L<level>/<members>" (the symbol itself comes before the '@').
static thread_local int t_prof_level = -1, t_prof_members = 0;
static std::string level_tag() {
  return t_prof_level < 0 ? std::string()
                          : "@L" + std::to_string(t_prof_level) + "/" + std::to_string(t_prof_members);
}
template <typename T>
static std::string kname(const Ctx* c, const char* base, const LMat<T>& m,
                         std::initializer_list<std::string> extra = {}) {
  if (!c->profiling) return std::string();
  std::vector<std::string> a{type_name<T>(), std::to_string(m.fmt),
                             std::to_string(m.fmt != kFmtCSR ? 1 : tpr_of(m.tpr))};
  for (const auto& e : extra) a.push_back(e);
  std::string s(base);
  const char* sep = "<";
  for (const auto& x : a) {
    s += sep;
    s += x;
    sep = ", ";
  }
  return s + ">" + level_tag();
}

template <typename T>
struct HalfL {
  Ctx* c;
  const LMat<T>& A;
  int r0, r1;
  const T *dinv, *B;
  GatherCF<T> X;
  const T* Xold;
  T* Xout;
  template <int FMT, int TPR>
  void go() const {
    if (r1 <= r0) return;
    hipLaunchKernelGGL((k_half<T, FMT, TPR>), rows_grid(r1 - launch_start<FMT>(r0), TPR, A.bs),
                       dim3(A.bs), 0, c->stream,
                       r0, r1, A.rp.get(), A.ci.get(), A.v.get(), dinv, B, X, Xold, Xout);
    MGD_CHECK_LAUNCH();
  }
};
template <typename T>
struct FHalf0L {
  Ctx* c;
  const LMat<T>& A;
  int r0, r1, nC;
  const T *dinv, *B, *XC;
  T* Xout;
  template <int FMT, int TPR>
  void go() const {
    if (r1 <= r0) return;
    hipLaunchKernelGGL((k_fhalf0<T, FMT, TPR>), rows_grid(r1 - launch_start<FMT>(r0), TPR, A.bs),
                       dim3(A.bs), 0, c->stream,
                       r0, r1, nC, A.rp.get(), A.ci.get(), A.v.get(), dinv, B, XC, Xout);
    MGD_CHECK_LAUNCH();
  }
};
template <typename T>
struct HalfOutL {
  Ctx* c;
  const LMat<T>& A;
  int nX, nC, nS;
  const T *dinv, *B;
  GatherCF<T> X;
  const T* XD;
  const int* perm;
  T* z;
  template <int FMT, int TPR>
  void go() const {
    if (nX <= 0) return;
    hipLaunchKernelGGL((k_half_out<T, FMT, TPR>), rows_grid(nX, TPR, A.bs), dim3(A.bs), 0, c->stream, 0,
                       nX, nC, nS, A.rp.get(), A.ci.get(), A.v.get(), dinv, B, X, XD, perm, z);
    MGD_CHECK_LAUNCH();
  }
};
template <typename T>
struct GsL {
  Ctx* c;
  const LMat<T>& A;
  int r0, n1, r2, n2;
  const T *dg, *B;
  T* X;
  template <int FMT, int TPR>
  void go() const {
    if (n1 + n2 <= 0) return;
    hipLaunchKernelGGL((k_gs<T, FMT, TPR>), rows_grid(n1 + n2, TPR, A.bs), dim3(A.bs), 0, c->stream, r0,
                       n1, r2, n2, A.rp.get(), A.ci.get(), A.v.get(), dg, B, X);
    MGD_CHECK_LAUNCH();
  }
};
template <typename T>
struct ResidL {
  Ctx* c;
  const LMat<T>& A;
  int nS;
  const T* B;
  GatherCF<T> X;
  T* R;
  template <int FMT, int TPR>
  void go() const {
    if (nS <= 0) return;
    hipLaunchKernelGGL((k_resid<T, FMT, TPR>), rows_grid(nS, TPR, A.bs), dim3(A.bs), 0, c->stream, 0, nS,
                       A.rp.get(), A.ci.get(), A.v.get(), B, X, R);
    MGD_CHECK_LAUNCH();
  }
};
template <typename T>
struct EntryResidL {
  Ctx* c;
  const LMat<T>& A;
  int nX, nS, nC;
  const int* perm;
  const T *dinv, *b, *z;
  T *B, *XC;
  bool pre;
  template <int FMT, int TPR>
  void go() const {
    if (nX <= 0) return;
    if (pre)
      hipLaunchKernelGGL((k_entry_resid<T, FMT, TPR, true>), rows_grid(nX, TPR, A.bs), dim3(A.bs), 0,
                         c->stream, 0, nX, nS, nC, A.rp.get(), A.ci.get(), A.v.get(), perm, dinv,
                         b, z, B, XC);
    else
      hipLaunchKernelGGL((k_entry_resid<T, FMT, TPR, false>), rows_grid(nX, TPR, A.bs), dim3(A.bs), 0,
                         c->stream, 0, nX, nS, nC, A.rp.get(), A.ci.get(), A.v.get(), perm, dinv,
                         b, z, B, XC);
    MGD_CHECK_LAUNCH();
  }
};
template <typename T>
struct RestrictL {
  Ctx* c;
  const LMat<T>& Wt;
  int nXn, nC, nCn;
  const int* cpos;
  const T *R, *dinv_n;
  T *Bn, *XCn;
  bool pre;
  template <int FMT, int TPR>
  void go() const {
    if (nXn <= 0) return;
    if (pre)
      hipLaunchKernelGGL((k_restrict<T, FMT, TPR, true>), rows_grid(nXn, TPR, Wt.bs), dim3(Wt.bs), 0,
                         c->stream, 0, nXn, nC, nCn, Wt.rp.get(), Wt.ci.get(), Wt.v.get(), cpos, R,
                         dinv_n, Bn, XCn);
    else
      hipLaunchKernelGGL((k_restrict<T, FMT, TPR, false>), rows_grid(nXn, TPR, Wt.bs), dim3(Wt.bs), 0,
                         c->stream, 0, nXn, nC, nCn, Wt.rp.get(), Wt.ci.get(), Wt.v.get(), cpos, R,
                         dinv_n, Bn, XCn);
    MGD_CHECK_LAUNCH();
  }
};
template <typename T>
struct ProlongL {
  Ctx* c;
  const LMat<T>& W;
  int nS, nC;
  const int* cmap;
  GatherCFD<T> E;
  T *XC, *XF;
  template <int FMT, int TPR>
  void go() const {
    if (nS <= 0) return;
    hipLaunchKernelGGL((k_prolong<T, FMT, TPR>), rows_grid(nS, TPR, W.bs), dim3(W.bs), 0, c->stream, 0,
                       nS, nC, W.rp.get(), W.ci.get(), W.v.get(), cmap, E, XC, XF);
    MGD_CHECK_LAUNCH();
  }
};

// algorithmic bytes per launch: every matrix entry (value + column), every
// per-row vector element read or written, and the gathered iterate once
template <typename T>
static double mat_bytes(const LMat<T>& m, long long nnz) {
  return (double)nnz * (sizeof(T) + (m.fmt == kFmtSELL16 ? 2 : 4));
}
// profiling scope of a launch that reads `nnz` entries of m over `rows` rows
// plus vec_bytes of vectors: stored-layout bytes, and the same launch priced
// as plain CSR (value and 4-byte column per entry, 4-byte row pointer per row)
template <typename T>
static ProfScope prof_level(Ctx* c, int cls, const LMat<T>& m, long long nnz, long long rows,
                            double vec_bytes, std::string name) {
  return ProfScope(c, cls, mat_bytes(m, nnz) + vec_bytes, std::move(name),
                   (double)nnz * (sizeof(T) + 4) + 4.0 * (double)rows + vec_bytes);
}
static inline int cls_of(int l, int cls0) { return l == 0 ? cls0 : KC_VCYCLE_COARSE; }

template <typename T>
static GatherCF<T> gather_cf(const T* xc, const T* xf, int nC) {
  return GatherCF<T>{xc, (ptrdiff_t)(xf - xc), nC};
}
template <typename T>
static GatherCFD<T> gather_cfd(const T* xc, const T* xf, const T* xd, int nC, int nS) {
  return GatherCFD<T>{xc, (ptrdiff_t)(xf - xc), (ptrdiff_t)(xd - xc), nC, nS};
}

template <typename T>
void Union<T>::vcycle(Ctx* c, T* z) {
  const int nl = (int)L.size();
  const size_t ts = sizeof(T);
  // current buffer (0: X0, 1: X1) of the C and the F region, per level
  std::vector<int> cc(nl, 0), cf(nl, 0);
  auto Xb = [&](int l, int which) -> T* { return which ? X1[l].get() : X0[l].get(); };
  t_prof_members = members;
  const int lt = tail_from >= 0 ? tail_from : nl;
  for (int l = 0; l < lt; ++l) {
    t_prof_level = l;
    ULevel<T>& lv = L[l];
    const int nF = lv.nS - lv.nC;
    // the C values of the first sweep were written with B (entry / restriction)
    if (lv.nS > 0) {
      for (int s = 0; s < n_pre; ++s) {
        if (s > 0) {  // C half of a later sweep
          ProfScope ps = prof_level(c, cls_of(l, KC_SMOOTH_L0), lv.A, lv.nnz_C, lv.nC,
                                    (double)lv.nC * 4 * ts + lv.nS * ts, kname(c, "k_half", lv.A));
          with_layout(lv.A.fmt, lv.A.tpr,
                      HalfL<T>{c, lv.A, 0, lv.nC, lv.dinv.get(), B[l].get(),
                               gather_cf<T>(Xb(l, cc[l]), Xb(l, cf[l]), lv.nC), Xb(l, cc[l]),
                               Xb(l, 1 - cc[l])});
          cc[l] = 1 - cc[l];
        }
        if (nF > 0) {
          if (s == 0) {
            ProfScope ps = prof_level(c, cls_of(l, KC_SMOOTH_L0), lv.A, lv.nnz_F, nF,
                                      (double)nF * 3 * ts + lv.nC * ts, kname(c, "k_fhalf0", lv.A));
            with_layout(lv.A.fmt, lv.A.tpr,
                        FHalf0L<T>{c, lv.A, lv.nC, lv.nS, lv.nC, lv.dinv.get(), B[l].get(),
                                   Xb(l, cc[l]), Xb(l, 1 - cf[l])});
          } else {
            ProfScope ps = prof_level(c, cls_of(l, KC_SMOOTH_L0), lv.A, lv.nnz_F, nF,
                                      (double)nF * 4 * ts + lv.nS * ts, kname(c, "k_half", lv.A));
            with_layout(lv.A.fmt, lv.A.tpr,
                        HalfL<T>{c, lv.A, lv.nC, lv.nS, lv.dinv.get(), B[l].get(),
                                 gather_cf<T>(Xb(l, cc[l]), Xb(l, cf[l]), lv.nC), Xb(l, cf[l]),
                                 Xb(l, 1 - cf[l])});
          }
          cf[l] = 1 - cf[l];
        }
      }
      if (n_pre == 0 && nF > 0) fill<T>(c, Xb(l, cf[l]) + lv.nC, (T)0, (size_t)nF);
      if (lv.nX_next > 0) {
        {
          ProfScope ps = prof_level(c, cls_of(l, KC_RESID_L0), lv.A, lv.A.nnz, lv.nS,
                                    (double)lv.nS * 3 * ts, kname(c, "k_resid", lv.A));
          with_layout(lv.A.fmt, lv.A.tpr,
                      ResidL<T>{c, lv.A, lv.nS, B[l].get(),
                                gather_cf<T>(Xb(l, cc[l]), Xb(l, cf[l]), lv.nC), R[l].get()});
        }
        const ULevel<T>& nx = L[l + 1];
        ProfScope ps = prof_level(c, cls_of(l, KC_TRANSFER_L0), lv.Wt, lv.Wt.nnz, lv.Wt.rows,
                                  (double)lv.nX_next * (4 + ts) + (double)nx.nC * 2 * ts +
                                      lv.nS * ts,
                                  kname(c, "k_restrict", lv.Wt, {n_pre > 0 ? "true" : "false"}));
        with_layout(lv.Wt.fmt, lv.Wt.tpr,
                    RestrictL<T>{c, lv.Wt, lv.nX_next, lv.nC, nx.nC, lv.cpos.get(), R[l].get(),
                                 nx.dinv.get(), B[l + 1].get(), Xb(l + 1, 0), n_pre > 0});
      }
    }
    if (!lv.dense.empty()) {
      ProfScope ps(c, KC_COARSE_SOLVE, 8.0 * lv.dense_entries + 2.0 * ts * (lv.nX - lv.nS),
                   ksym(c, "k_dense", {type_name<T>()}));
      dim3 grid(cdiv(lv.dense_max_n, 64), (unsigned)lv.dense.size());
      hipLaunchKernelGGL(k_dense<T>, grid, dim3(256), 0, c->stream,
                         (const DenseDev*)lv.dense_dev.get(), (const T*)B[l].get(), X0[l].get());
      MGD_CHECK_LAUNCH();
    }
  }
  if (lt < nl) {  // levels lt .. nl-1, down and up, in one launch
    t_prof_level = lt;
    ProfScope ps(c, KC_VCYCLE_COARSE, tail_bytes, ksym(c, "k_tail", {type_name<T>()}) + level_tag(),
                 tail_bytes_csr);
    hipLaunchKernelGGL(k_tail<T>, dim3(tail_blocks), dim3(kTailThreads), 0, c->stream,
                       (const TailOp<T>*)tail_ops.get(), tail_nops, tail_sync.get(), c->err_flag());
    MGD_CHECK_LAUNCH();
    cc[lt] = tail_cc;
    cf[lt] = tail_cf;
  }
  for (int l = lt - 1; l >= 0; --l) {
    t_prof_level = l;
    ULevel<T>& lv = L[l];
    const int nF = lv.nS - lv.nC;
    if (lv.nS > 0 && lv.nX_next > 0) {
      const ULevel<T>& nx = L[l + 1];
      ProfScope ps = prof_level(c, cls_of(l, KC_TRANSFER_L0), lv.W, lv.W.nnz, lv.W.rows,
                                (double)lv.nC * 4 + lv.nS * 2.0 * ts + (double)lv.nX_next * ts,
                                kname(c, "k_prolong", lv.W));
      with_layout(lv.W.fmt, lv.W.tpr,
                  ProlongL<T>{c, lv.W, lv.nS, lv.nC, lv.cmap.get(),
                              gather_cfd<T>(Xb(l + 1, cc[l + 1]), Xb(l + 1, cf[l + 1]),
                                            X0[l + 1].get(), nx.nC, nx.nS),
                              Xb(l, cc[l]), Xb(l, cf[l])});
    }
    const bool last_out = (l == 0);
    if (lv.nS > 0) {
      for (int s = 0; s < n_post; ++s) {
        if (nF > 0) {
          ProfScope ps = prof_level(c, cls_of(l, KC_SMOOTH_L0), lv.A, lv.nnz_F, nF,
                                    (double)nF * 4 * ts + lv.nS * ts, kname(c, "k_half", lv.A));
          with_layout(lv.A.fmt, lv.A.tpr,
                      HalfL<T>{c, lv.A, lv.nC, lv.nS, lv.dinv.get(), B[l].get(),
                               gather_cf<T>(Xb(l, cc[l]), Xb(l, cf[l]), lv.nC), Xb(l, cf[l]),
                               Xb(l, 1 - cf[l])});
          cf[l] = 1 - cf[l];
        }
        if (last_out && z && s == n_post - 1) {  // final C half writes the natural result
          ProfScope ps = prof_level(c, KC_SMOOTH_L0, lv.A, lv.nnz_C, lv.nC,
                                    (double)lv.nC * 3 * ts + lv.nS * ts + (double)lv.nX * (4 + ts),
                                    kname(c, "k_half_out", lv.A));
          with_layout(lv.A.fmt, lv.A.tpr,
                      HalfOutL<T>{c, lv.A, lv.nX, lv.nC, lv.nS, lv.dinv.get(), B[l].get(),
                                  gather_cf<T>(Xb(l, cc[l]), Xb(l, cf[l]), lv.nC), X0[l].get(),
                                  lv.perm.get(), z});
          return;
        }
        ProfScope ps = prof_level(c, cls_of(l, KC_SMOOTH_L0), lv.A, lv.nnz_C, lv.nC,
                                  (double)lv.nC * 4 * ts + lv.nS * ts, kname(c, "k_half", lv.A));
        with_layout(lv.A.fmt, lv.A.tpr,
                    HalfL<T>{c, lv.A, 0, lv.nC, lv.dinv.get(), B[l].get(),
                             gather_cf<T>(Xb(l, cc[l]), Xb(l, cf[l]), lv.nC), Xb(l, cc[l]),
                             Xb(l, 1 - cc[l])});
        cc[l] = 1 - cc[l];
      }
    }
    if (last_out && !z) {  // the result stays in stored order
      out_cc = cc[0];
      out_cf = cf[0];
      return;
    }
    if (last_out) {  // no post-smoothing (or no stored rows): copy out
      hipLaunchKernelGGL(k_out<T>, dim3(cdiv(lv.nX, 256)), dim3(256), 0, c->stream, lv.nX,
                         gather_cfd<T>(Xb(0, cc[0]), Xb(0, cf[0]), X0[0].get(), lv.nC, lv.nS),
                         (const int*)lv.perm.get(), z);
      MGD_CHECK_LAUNCH();
    }
  }
}

// Levels from which the persistent tail takes over: the first level from
// which every level has at most MGD_TAIL_ROWS extended rows (default
// kTailRows = 0: off, the per-level launches measure faster on gfx950, where
// the barrier's device-scope release and acquire write back and invalidate
// the L2 of the workgroup's chiplet at every phase).  Workgroups:
// MGD_TAIL_BLOCKS (default kTailBlocks), capped by what the device holds
// resident at once.
constexpr int kTailRows = 0;
constexpr int kTailBlocks = 256;
static long long env_ll(const char* name, long long dflt) {
  const char* e = std::getenv(name);
  return e && *e ? std::atoll(e) : dflt;
}

// The phase table of vcycle() for levels >= tail_from, recorded with the same
// buffer choices (the two iterate buffers of every level start at X0 in each
// cycle, so the table is the same for every cycle).
template <typename T>
void Union<T>::build_tail(Ctx* c) {
  tail_from = -1;
  const int nl = (int)L.size();
  const long long rows = env_ll("MGD_TAIL_ROWS", kTailRows);
  if (gs || n_pre < 1 || rows <= 0 || nl < 2) return;
  int lt = nl;
  while (lt > 1 && L[lt - 1].nX <= rows) --lt;
  if (lt >= nl) return;
  std::vector<int> cc(nl, 0), cf(nl, 0);
  auto Xb = [&](int l, int which) -> T* { return which ? X1[l].get() : X0[l].get(); };
  std::vector<TailOp<T>> ops;
  double bytes = 0, bytes_csr = 0;
  const size_t ts = sizeof(T);
  auto mat_op = [&](int kind, const LMat<T>& m, int r0, int r1, long long nnz, double vec) {
    TailOp<T> o{};
    o.kind = kind;
    o.fmt = m.fmt;
    o.tpr = m.fmt == kFmtCSR ? tpr_of(m.tpr) : 1;
    o.r0 = r0;
    o.r1 = r1;
    o.rp = m.rp.get();
    o.ci = m.ci.get();
    o.v = m.v.get();
    bytes += mat_bytes(m, nnz) + vec;
    bytes_csr += (double)nnz * (ts + 4) + 4.0 * (r1 - r0) + vec;
    return o;
  };
  auto gather = [&](TailOp<T>& o, int l) {
    o.xc = Xb(l, cc[l]);
    o.f_minus_c = Xb(l, cf[l]) - Xb(l, cc[l]);
    o.nC = L[l].nC;
  };
  for (int l = lt; l < nl; ++l) {  // down: the same steps as vcycle()
    ULevel<T>& lv = L[l];
    const int nF = lv.nS - lv.nC;
    if (lv.nS > 0) {
      for (int s = 0; s < n_pre; ++s) {
        if (s > 0) {
          if (lv.nC > 0) {
            TailOp<T> o = mat_op(kTopHalf, lv.A, 0, lv.nC, lv.nnz_C, (double)lv.nC * 4 * ts + lv.nS * ts);
            gather(o, l);
            o.dinv = lv.dinv.get();
            o.B = B[l].get();
            o.xold = Xb(l, cc[l]);
            o.out = Xb(l, 1 - cc[l]);
            ops.push_back(o);
          }
          cc[l] = 1 - cc[l];
        }
        if (nF > 0) {
          TailOp<T> o = mat_op(s == 0 ? kTopFHalf0 : kTopHalf, lv.A, lv.nC, lv.nS, lv.nnz_F,
                               (double)nF * (s == 0 ? 3 : 4) * ts + (s == 0 ? lv.nC : lv.nS) * ts);
          gather(o, l);
          o.dinv = lv.dinv.get();
          o.B = B[l].get();
          o.xold = Xb(l, cf[l]);
          o.out = Xb(l, 1 - cf[l]);
          ops.push_back(o);
          cf[l] = 1 - cf[l];
        }
      }
      if (lv.nX_next > 0) {
        TailOp<T> o = mat_op(kTopResid, lv.A, 0, lv.nS, lv.A.nnz, (double)lv.nS * 3 * ts);
        gather(o, l);
        o.B = B[l].get();
        o.out = R[l].get();
        ops.push_back(o);
        const ULevel<T>& nx = L[l + 1];
        TailOp<T> q = mat_op(kTopRestrict, lv.Wt, 0, lv.nX_next, lv.Wt.nnz,
                             (double)lv.nX_next * (4 + ts) + (double)nx.nC * 2 * ts + lv.nS * ts);
        q.nC = lv.nC;
        q.nCn = nx.nC;
        q.pre = 1;
        q.map = lv.cpos.get();
        q.B = R[l].get();
        q.dinv = nx.dinv.get();
        q.out = B[l + 1].get();
        q.out2 = X0[l + 1].get();
        ops.push_back(q);
      }
    }
    if (!lv.dense.empty()) {
      TailOp<T> o{};
      o.kind = kTopDense;
      o.dense = (const DenseDev*)lv.dense_dev.get();
      o.ndense = (int)lv.dense.size();
      o.dchunks = cdiv(lv.dense_max_n, 64);
      o.B = B[l].get();
      o.out = X0[l].get();
      bytes += 8.0 * lv.dense_entries + 2.0 * ts * (lv.nX - lv.nS);
      bytes_csr += 8.0 * lv.dense_entries + 2.0 * ts * (lv.nX - lv.nS);
      ops.push_back(o);
    }
  }
  for (int l = nl - 1; l >= lt; --l) {  // up
    ULevel<T>& lv = L[l];
    const int nF = lv.nS - lv.nC;
    if (lv.nS > 0 && lv.nX_next > 0) {
      const ULevel<T>& nx = L[l + 1];
      TailOp<T> o = mat_op(kTopProlong, lv.W, 0, lv.nS, lv.W.nnz,
                           (double)lv.nC * 4 + lv.nS * 2.0 * ts + (double)lv.nX_next * ts);
      o.xc = Xb(l + 1, cc[l + 1]);
      o.f_minus_c = Xb(l + 1, cf[l + 1]) - Xb(l + 1, cc[l + 1]);
      o.d_minus_c = X0[l + 1].get() - Xb(l + 1, cc[l + 1]);
      o.nC = nx.nC;
      o.nS = nx.nS;
      o.nCn = lv.nC;
      o.map = lv.cmap.get();
      o.out2 = Xb(l, cc[l]);
      o.out = Xb(l, cf[l]);
      ops.push_back(o);
    }
    if (lv.nS > 0) {
      for (int s = 0; s < n_post; ++s) {
        if (nF > 0) {
          TailOp<T> o = mat_op(kTopHalf, lv.A, lv.nC, lv.nS, lv.nnz_F, (double)nF * 4 * ts + lv.nS * ts);
          gather(o, l);
          o.dinv = lv.dinv.get();
          o.B = B[l].get();
          o.xold = Xb(l, cf[l]);
          o.out = Xb(l, 1 - cf[l]);
          ops.push_back(o);
          cf[l] = 1 - cf[l];
        }
        if (lv.nC > 0) {
          TailOp<T> o = mat_op(kTopHalf, lv.A, 0, lv.nC, lv.nnz_C, (double)lv.nC * 4 * ts + lv.nS * ts);
          gather(o, l);
          o.dinv = lv.dinv.get();
          o.B = B[l].get();
          o.xold = Xb(l, cc[l]);
          o.out = Xb(l, 1 - cc[l]);
          ops.push_back(o);
        }
        cc[l] = 1 - cc[l];
      }
    }
  }
  if (ops.empty()) return;
  // workgroups resident at once on the whole device
  int dev = 0, cus = 0, per_cu = 0;
  MGD_HIP(hipGetDevice(&dev));
  MGD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  MGD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tail<T>, kTailThreads, 0));
  const long long want = env_ll("MGD_TAIL_BLOCKS", kTailBlocks);
  tail_blocks = (int)std::max(1LL, std::min(want, (long long)cus * std::max(per_cu, 1)));
  tail_ops.alloc(c, ops.size());
  copy_h2d(c, tail_ops.get(), ops.data(), ops.size());
  tail_sync.alloc(c, 2 * kTailSyncStride);
  fill<unsigned>(c, tail_sync.get(), 0u, 2 * kTailSyncStride);
  tail_nops = (int)ops.size();
  tail_cc = cc[lt];
  tail_cf = cf[lt];
  tail_bytes = bytes;
  tail_bytes_csr = bytes_csr;
  tail_from = lt;
}

template <typename T>
void Union<T>::gs_sweep(Ctx* c, int l, bool descending) {
  ULevel<T>& lv = L[l];
  const int nc = (int)lv.cranges.size();
  for (int q = 0; q < nc; ++q) {
    const auto& r = lv.cranges[descending ? nc - 1 - q : q];
    const int n1 = r[1] - r[0], n2 = r[3] - r[2];
    if (n1 + n2 == 0) continue;
    ProfScope ps(c, cls_of(l, KC_SMOOTH_L0), 0.0, kname(c, "k_gs", lv.A));
    with_layout(lv.A.fmt, lv.A.tpr,
                GsL<T>{c, lv.A, r[0], n1, r[2], n2, lv.dgs.get(), B[l].get(), X0[l].get()});
  }
}

// V-cycle with multicolour Gauss-Seidel: one iterate buffer per level, updated
// in place colour by colour (ascending going down, descending going up)
template <typename T>
void Union<T>::vcycle_gs(Ctx* c, T* z) {
  const int nl = (int)L.size();
  for (int l = 0; l < nl; ++l) {
    ULevel<T>& lv = L[l];
    const int nF = lv.nS - lv.nC;
    if (lv.nS > 0) {
      if (nF > 0) fill<T>(c, X0[l].get() + lv.nC, (T)0, (size_t)nF);  // C part zeroed with B
      for (int s = 0; s < n_pre; ++s) gs_sweep(c, l, false);
      if (lv.nX_next > 0) {
        {
          ProfScope ps(c, cls_of(l, KC_RESID_L0), 0.0, kname(c, "k_resid", lv.A));
          with_layout(lv.A.fmt, lv.A.tpr,
                      ResidL<T>{c, lv.A, lv.nS, B[l].get(),
                                gather_cf<T>(X0[l].get(), X0[l].get(), lv.nC), R[l].get()});
        }
        const ULevel<T>& nx = L[l + 1];
        ProfScope ps(c, cls_of(l, KC_TRANSFER_L0), 0.0, kname(c, "k_restrict", lv.Wt, {"false"}));
        with_layout(lv.Wt.fmt, lv.Wt.tpr,
                    RestrictL<T>{c, lv.Wt, lv.nX_next, lv.nC, nx.nC, lv.cpos.get(), R[l].get(),
                                 nx.dinv.get(), B[l + 1].get(), X0[l + 1].get(), false});
      }
    }
    if (!lv.dense.empty()) {
      ProfScope ps(c, KC_COARSE_SOLVE, 8.0 * lv.dense_entries, ksym(c, "k_dense", {type_name<T>()}));
      dim3 grid(cdiv(lv.dense_max_n, 64), (unsigned)lv.dense.size());
      hipLaunchKernelGGL(k_dense<T>, grid, dim3(256), 0, c->stream,
                         (const DenseDev*)lv.dense_dev.get(), (const T*)B[l].get(), X0[l].get());
      MGD_CHECK_LAUNCH();
    }
  }
  for (int l = nl - 1; l >= 0; --l) {
    ULevel<T>& lv = L[l];
    if (lv.nS > 0 && lv.nX_next > 0) {
      const ULevel<T>& nx = L[l + 1];
      ProfScope ps(c, cls_of(l, KC_TRANSFER_L0), 0.0, kname(c, "k_prolong", lv.W));
      with_layout(lv.W.fmt, lv.W.tpr,
                  ProlongL<T>{c, lv.W, lv.nS, lv.nC, lv.cmap.get(),
                              gather_cfd<T>(X0[l + 1].get(), X0[l + 1].get(), X0[l + 1].get(),
                                            nx.nC, nx.nS),
                              X0[l].get(), X0[l].get()});
    }
    if (lv.nS > 0)
      for (int s = 0; s < n_post; ++s) gs_sweep(c, l, true);
  }
  ULevel<T>& l0 = L[0];
  hipLaunchKernelGGL(k_out<T>, dim3(cdiv(l0.nX, 256)), dim3(256), 0, c->stream, l0.nX,
                     gather_cfd<T>(X0[0].get(), X0[0].get(), X0[0].get(), l0.nC, l0.nS),
                     (const int*)l0.perm.get(), z);
  MGD_CHECK_LAUNCH();
}

template <typename T>
void Union<T>::apply_seg(Ctx* c, int N, const SegIn* tab, const double* r, const T* w, T* z) {
  ULevel<T>& l0 = L[0];
  MGD_REQUIRE(N > 0 && (long long)N * members == l0.nX, "apply_seg: rows do not match the union");
  MGD_REQUIRE(z || (!gs && tail_from != 0), "apply_seg: stored-order result needs level-0 launches");
  const bool pre = n_pre > 0 && !gs;
  {
    // iperm, r and the coefficients (FP64), w, d^-1 on C rows, B and X_C written
    ProfScope ps(c, KC_TRANSFER_L0,
                 (double)l0.nX * (4 + 16 + 2.0 * sizeof(T)) + l0.nC * 2.0 * sizeof(T),
                 ksym(c, "k_entry_nat", {type_name<T>(), pre ? "true" : "false"}));
    const dim3 grid(cdiv(N, 256), members);
    if (pre)
      hipLaunchKernelGGL((k_entry_nat<T, true>), grid, dim3(256), 0, c->stream, N, l0.nC,
                         (const int*)l0.iperm.get(), (const T*)l0.dinv_nat.get(), tab, r, w,
                         B[0].get(), X0[0].get());
    else
      hipLaunchKernelGGL((k_entry_nat<T, false>), grid, dim3(256), 0, c->stream, N, l0.nC,
                         (const int*)l0.iperm.get(), (const T*)l0.dinv_nat.get(), tab, r, w,
                         B[0].get(), X0[0].get());
    MGD_CHECK_LAUNCH();
  }
  if (gs)
    vcycle_gs(c, z);
  else
    vcycle(c, z);
  t_prof_level = -1;
}

template <typename T>
StoredOut<T> Union<T>::stored_out() const {
  const ULevel<T>& l0 = L[0];
  return {l0.iperm.get(), (out_cc ? X1[0] : X0[0]).get(), (out_cf ? X1[0] : X0[0]).get(),
          X0[0].get(), l0.nC, l0.nS};
}

template <typename T>
void Union<T>::apply(Ctx* c, const T* bvec, T* z, int cycles) {
  ULevel<T>& l0 = L[0];
  const bool pre = n_pre > 0 && !gs;  // first-sweep C values (CF-l1-Jacobi only)
  {
    ProfScope ps(c, KC_TRANSFER_L0, (double)l0.nX * (4 + 2.0 * sizeof(T)) + l0.nC * 2.0 * sizeof(T),
                 ksym(c, "k_entry", {type_name<T>(), pre ? "true" : "false"}));
    if (pre)
      hipLaunchKernelGGL((k_entry<T, true>), dim3(cdiv(l0.nX, 256)), dim3(256), 0, c->stream,
                         l0.nX, l0.nC, (const int*)l0.perm.get(), (const T*)l0.dinv.get(), bvec,
                         B[0].get(), X0[0].get());
    else
      hipLaunchKernelGGL((k_entry<T, false>), dim3(cdiv(l0.nX, 256)), dim3(256), 0, c->stream,
                         l0.nX, l0.nC, (const int*)l0.perm.get(), (const T*)l0.dinv.get(), bvec,
                         B[0].get(), X0[0].get());
    MGD_CHECK_LAUNCH();
  }
  if (gs)
    vcycle_gs(c, z);
  else
    vcycle(c, z);
  for (int k = 1; k < cycles; ++k) {
    {
      ProfScope ps = prof_level(c, KC_RESID_L0, l0.A, l0.A.nnz, l0.nS,
                                (double)l0.nX * (8 + 3.0 * sizeof(T)),
                                kname(c, "k_entry_resid", l0.A, {pre ? "true" : "false"}));
      with_layout(l0.A.fmt, l0.A.tpr,
                  EntryResidL<T>{c, l0.A, l0.nX, l0.nS, l0.nC, l0.perm.get(), l0.dinv.get(), bvec,
                                 z, B[0].get(), X0[0].get(), pre});
    }
    if (gs)
      vcycle_gs(c, t1.get());
    else
      vcycle(c, t1.get());
    hipLaunchKernelGGL(k_axpy_t<T>, dim3(cdiv(n0, 256)), dim3(256), 0, c->stream, n0,
                       (const T*)t1.get(), z);
    MGD_CHECK_LAUNCH();
  }
  t_prof_level = -1;
}

template <typename T>
double Union<T>::bytes_per_vcycle() const {
  const double ts = sizeof(T);
  double s = 0;
  for (size_t l = 0; l < L.size(); ++l) {
    const auto& lv = L[l];
    const double nF = lv.nS - lv.nC;
    if (lv.nS > 0) {
      s += mat_bytes(lv.A, lv.nnz_F) * (n_pre + n_post) + mat_bytes(lv.A, lv.nnz_C) * (n_pre + n_post - 1);
      s += (nF * 4 * ts + lv.nS * ts) * (n_pre + n_post) +
           (lv.nC * 4 * ts + lv.nS * ts) * (n_pre + n_post - 1);
      if (lv.nX_next > 0) {
        s += mat_bytes(lv.A, lv.A.nnz) + lv.nS * 3 * ts;
        s += mat_bytes(lv.Wt, lv.Wt.nnz) + lv.nX_next * (4 + ts) + lv.nS * ts;
        s += mat_bytes(lv.W, lv.W.nnz) + lv.nC * 4.0 + lv.nS * 2.0 * ts + lv.nX_next * ts;
      }
    }
    s += 8.0 * lv.dense_entries;
  }
  return s;
}

static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune;
static bool g_tune_loaded = false;

static std::string tune_key(long long rows, long long nnz, int maxrow, bool fp32,
                            const char* kind) {
  std::ostringstream o;
  o << (fp32 ? "f32:" : "f64:") << kind << rows << ":" << nnz << ":" << maxrow;
  return o.str();
}
static void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("MGD_AUTOTUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  std::string tok;
  // format: {"key": value, ...}
  std::string all((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  size_t p = 0;
  while ((p = all.find('"', p)) != std::string::npos) {
    size_t q = all.find('"', p + 1);
    if (q == std::string::npos) break;
    std::string key = all.substr(p + 1, q - p - 1);
    size_t colon = all.find(':', q);
    if (colon == std::string::npos) break;
    g_tune[key] = std::atoi(all.c_str() + colon + 1);
    p = colon + 1;
  }
}
static void tune_save_locked() {
  const char* path = std::getenv("MGD_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream f(path);
  f << "{";
  bool first = true;
  for (auto& kv : g_tune) {
    f << (first ? "" : ",") << "\n  \"" << kv.first << "\": " << kv.second;
    first = false;
  }
  f << "\n}\n";
}
int autotune_lookup(long long rows, long long nnz, int maxrow, bool fp32, const char* kind) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(tune_key(rows, nnz, maxrow, fp32, kind));
  return it == g_tune.end() ? 0 : it->second;
}
void autotune_store(long long rows, long long nnz, int maxrow, bool fp32, int tpr,
                    const char* kind) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load_locked();
  g_tune[tune_key(rows, nnz, maxrow, fp32, kind)] = tpr;
  tune_save_locked();
}

__global__ void k_max_row(int n, const int* __restrict__ rp, int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int m = i < n ? rp[i + 1] - rp[i] : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(out, m);
}

// ---------------------------------------------------------------------------
// stored-order finalisation and level layouts
// ---------------------------------------------------------------------------
// SELL slice widths (64 x the longest row of each 64-row slice)
__global__ void k_slice_width(int rows, const int* __restrict__ rp, int* __restrict__ w64) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int ns = (rows + 63) / 64;
  if (s >= ns) return;
  int m = 0;
  const int r1 = min(rows, 64 * s + 64);
  for (int r = 64 * s; r < r1; ++r) m = max(m, rp[r + 1] - rp[r]);
  w64[s] = 64 * m;
}
template <typename T>
__global__ void k_sell_fill(int rows, const int* __restrict__ rp, const int* __restrict__ ci,
                            const double* __restrict__ v, const int* __restrict__ off,
                            int self_pad, int* __restrict__ sci, T* __restrict__ sv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int o = off[r >> 6] + (r & 63), w = (off[(r >> 6) + 1] - off[r >> 6]) >> 6;
  const int e0 = rp[r], len = rp[r + 1] - e0;
  const int pad = self_pad ? r : 0;  // padding reads a defined element with weight zero
  for (int e = 0; e < w; ++e) {
    const bool in = e < len;
    sci[o + 64 * e] = in ? ci[e0 + e] : pad;
    sv[o + 64 * e] = in ? (T)v[e0 + e] : (T)0;
  }
}

// Test override: MGD_SELL16_SPAN lowers the column span a slice side may have
// in the 16-bit layout (so that small systems get 32-bit slices too).
static int sell16_span() {
  const char* e = std::getenv("MGD_SELL16_SPAN");
  const int d = 0x7fff;
  return e && *e ? std::min(d, std::max(0, std::atoi(e))) : d;
}

// SELL16 bases of slice s from the real entries of its rows (CSR M): the
// smallest column below `split` and the smallest at or above it (0 without
// one); a side spanning more than `span` (<= 2^15 - 1) columns makes the
// slice keep 32-bit columns (F base -1).  units[s]: the slice's code size in
// 16-bit units.
__global__ void k_sell16_bases(int rows, const int* __restrict__ rp, const int* __restrict__ ci,
                               int split, int span, const int* __restrict__ off,
                               int* __restrict__ rp4, int* __restrict__ units) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int ns = (rows + 63) / 64;
  if (s >= ns) return;
  int cmin = INT_MAX, cmax = -1, fmin = INT_MAX, fmax = -1;
  const int r1 = min(rows, 64 * s + 64);
  for (int r = 64 * s; r < r1; ++r)
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
      const int j = ci[e];
      if (j < split) {
        cmin = min(cmin, j);
        cmax = max(cmax, j);
      } else {
        fmin = min(fmin, j);
        fmax = max(fmax, j);
      }
    }
  const bool wide = (cmax >= 0 && cmax - cmin > span) || (fmax >= 0 && fmax - fmin > span);
  rp4[4 * s] = off[s];
  rp4[4 * s + 2] = cmax >= 0 ? cmin : 0;
  rp4[4 * s + 3] = wide ? -1 : (fmax >= 0 ? fmin : 0);
  units[s] = (off[s + 1] - off[s]) * (wide ? 2 : 1);
  if (s == ns - 1) rp4[4 * ns] = off[ns];
}
__global__ void k_sell16_coff(int ns, const int* __restrict__ coff, int* __restrict__ rp4) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s <= ns) rp4[4 * s + 1] = coff[s];
}
// codes of row r: column - C base below the split, (column - F base) | 2^15
// at or above it, or the column itself in a 32-bit slice; padding elements
// get code 0 (the C base, or column 0, with weight zero)
__global__ void k_sell16_encode(int rows, const int* __restrict__ rp, const int* __restrict__ ci,
                                int split, const int* __restrict__ rp4, uint16_t* __restrict__ c16) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int s4 = 4 * (r >> 6);
  const int w = (rp4[s4 + 4] - rp4[s4]) >> 6;
  const int cb = rp4[s4 + 2], fb = rp4[s4 + 3];
  const int e0 = rp[r], len = rp[r + 1] - e0;
  if (fb < 0) {
    int* c32 = reinterpret_cast<int*>(c16) + (rp4[s4 + 1] >> 1) + (r & 63);
    for (int q = 0; q < w; ++q) c32[64 * q] = q < len ? ci[e0 + q] : 0;
    return;
  }
  const int oc = rp4[s4 + 1] + (r & 63);
  for (int q = 0; q < w; ++q) {
    unsigned code = 0;
    if (q < len) {
      const int j = ci[e0 + q];
      code = j < split ? (unsigned)(j - cb) : (0x8000u | (unsigned)(j - fb));
    }
    c16[oc + 64 * q] = (uint16_t)code;
  }
}
// every real element decodes to its CSR column, every padding element to a
// column inside [0, ncols)
__global__ void k_sell16_check(int rows, int ncols, const int* __restrict__ rp,
                               const int* __restrict__ ci, const int* __restrict__ rp4,
                               const int* __restrict__ codes, int* __restrict__ err) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  int o, oc, w, cb, fb;
  sell_slice<kFmtSELL16>(rp4, r, o, oc, w, cb, fb);
  const int e0 = rp[r], len = rp[r + 1] - e0;
  for (int q = 0; q < w; ++q) {
    const int j = fb >= 0 ? sell_col<true>(codes, oc + 64 * q, cb, fb)
                          : sell_col<false>(codes, oc + 64 * q, cb, fb);
    if (q < len ? j != ci[e0 + q] : (j < 0 || j >= ncols)) atomicOr(err, 4);
  }
}

// CSR (FP64 values) -> layout `fmt` with values in T; `self_pad` pads SELL rows
// with their own index as column (square stored-order matrices), else column 0.
// A SELL result becomes SELL16 when split16 >= 0 and every slice fits.
template <typename T>
static void to_layout(Ctx* c, const Csr<double>& M, int fmt, int tpr, bool self_pad,
                      LMat<T>& out, int split16 = -1) {
  out.rows = M.n_rows;
  out.nnz = M.nnz;
  out.fmt = fmt;
  out.tpr = tpr;
  if (fmt == kFmtCSR || M.n_rows == 0) {
    out.fmt = kFmtCSR;
    out.stored = M.nnz;
    out.rp.alloc(c, (size_t)M.n_rows + 1);
    copy_d2d(c, out.rp.get(), M.rp.get(), (size_t)M.n_rows + 1);
    out.ci.alloc(c, (size_t)std::max(M.nnz, 1));
    copy_d2d(c, out.ci.get(), M.ci.get(), (size_t)M.nnz);
    out.v.alloc(c, (size_t)std::max(M.nnz, 1));
    cast_copy<T, double>(c, out.v.get(), M.v.get(), (size_t)M.nnz, KC_VEC);
    c->sync();
    return;
  }
  const int ns = cdiv(M.n_rows, 64);
  DBuf<int> w64(c, (size_t)ns);
  hipLaunchKernelGGL(k_slice_width, dim3(cdiv(ns, 256)), dim3(256), 0, c->stream, M.n_rows,
                     (const int*)M.rp.get(), w64.get());
  MGD_CHECK_LAUNCH();
  out.rp.alloc(c, (size_t)ns + 1);
  out.stored = exclusive_scan_total(c, w64.get(), out.rp.get(), ns);
  out.ci.alloc(c, (size_t)std::max(out.stored, 1LL));
  out.v.alloc(c, (size_t)std::max(out.stored, 1LL));
  hipLaunchKernelGGL(k_sell_fill<T>, dim3(cdiv(M.n_rows, 256)), dim3(256), 0, c->stream,
                     M.n_rows, (const int*)M.rp.get(), (const int*)M.ci.get(),
                     (const double*)M.v.get(), (const int*)out.rp.get(), self_pad ? 1 : 0,
                     out.ci.get(), out.v.get());
  MGD_CHECK_LAUNCH();
  c->sync();
  if (split16 < 0 || M.nnz == 0) return;
  DBuf<int> rp4(c, 4 * (size_t)ns + 2), units(c, (size_t)ns), coff(c, (size_t)ns + 1);
  hipLaunchKernelGGL(k_sell16_bases, dim3(cdiv(ns, 256)), dim3(256), 0, c->stream, M.n_rows,
                     (const int*)M.rp.get(), (const int*)M.ci.get(), split16, sell16_span(),
                     (const int*)out.rp.get(), rp4.get(), units.get());
  MGD_CHECK_LAUNCH();
  const long long total = exclusive_scan_total(c, units.get(), coff.get(), ns);
  hipLaunchKernelGGL(k_sell16_coff, dim3(cdiv(ns + 1, 256)), dim3(256), 0, c->stream, ns,
                     (const int*)coff.get(), rp4.get());
  MGD_CHECK_LAUNCH();
  DBuf<int> codes(c, (size_t)std::max(1LL, (total + 1) / 2));
  hipLaunchKernelGGL(k_sell16_encode, dim3(cdiv(M.n_rows, 256)), dim3(256), 0, c->stream,
                     M.n_rows, (const int*)M.rp.get(), (const int*)M.ci.get(), split16,
                     (const int*)rp4.get(), reinterpret_cast<uint16_t*>(codes.get()));
  MGD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sell16_check, dim3(cdiv(M.n_rows, 256)), dim3(256), 0, c->stream,
                     M.n_rows, M.n_cols, (const int*)M.rp.get(), (const int*)M.ci.get(),
                     (const int*)rp4.get(), (const int*)codes.get(), c->err_flag());
  MGD_CHECK_LAUNCH();
  c->check_device_errors("16-bit sliced layout");
  out.rp = std::move(rp4);
  out.ci = std::move(codes);
  out.fmt = kFmtSELL16;
}
// padded size of the SELL layout of M (host-side estimate through the device widths)
static long long sell_stored(Ctx* c, const Csr<double>& M) {
  if (M.n_rows == 0) return 0;
  const int ns = cdiv(M.n_rows, 64);
  DBuf<int> w64(c, (size_t)ns), tmp(c, (size_t)ns + 1);
  hipLaunchKernelGGL(k_slice_width, dim3(cdiv(ns, 256)), dim3(256), 0, c->stream, M.n_rows,
                     (const int*)M.rp.get(), w64.get());
  MGD_CHECK_LAUNCH();
  return exclusive_scan_total(c, w64.get(), tmp.get(), ns);
}

template <typename T>
static void tune_layout(Ctx* c, ULevel<T>& lv, const Csr<double>& A, int autotune, bool fp32);
template <typename T>
static void tune_restrict(Ctx* c, const ULevel<T>& lv, int nS, int nC, int nCn,
                          const Csr<double>& Wt, LMat<T>& out, int autotune, bool fp32);

constexpr long long kFillLanes = 1 << 17;  // lanes that keep all compute units busy
constexpr int kSellMinRows = 1 << 17;
// Test overrides: MGD_SELL_MIN_ROWS lowers the row count from which sliced
// layouts are considered (so that small systems exercise them), MGD_SELL16=0
// keeps sliced layouts at 32-bit columns.
static long long sell_min_rows() {
  const char* e = std::getenv("MGD_SELL_MIN_ROWS");
  return e && *e ? std::max(1LL, std::atoll(e)) : (long long)kSellMinRows;
}
// Matrices with fewer rows keep the default layout rule: their launches are
// latency bound, and timing them back to back with their data in cache does
// not rank the layouts as their launches inside a cycle do.  MGD_TUNE_MIN_ROWS
// (tests) lowers the bound.
constexpr int kTuneMinRows = 1 << 17;
static long long tune_min_rows() {
  const char* e = std::getenv("MGD_TUNE_MIN_ROWS");
  return e && *e ? std::max(1LL, std::atoll(e)) : (long long)kTuneMinRows;
}
static bool sell16_enabled() {
  const char* e = std::getenv("MGD_SELL16");
  return !(e && e[0] == '0');
}
// lanes per row so that a small matrix still spreads over the device
static int small_level_tpr(long long rows, double avg) {
  int t = 1;
  while (t < 64 && rows * t < kFillLanes && t < avg) t *= 2;
  return t;
}
// interpolation / restriction layout: SELL for large matrices with little
// padding (sell_entries: the SELL layout's stored entries), otherwise CSR with
// enough lanes per row; the result is kTuneSell (1000) or the lanes per row
static int transfer_default(const Csr<double>& M, long long sell_entries) {
  const double avg = M.n_rows ? (double)M.nnz / M.n_rows : 1.0;
  if (M.nnz > 0 && M.n_rows >= sell_min_rows() && sell_entries <= (long long)(1.5 * M.nnz))
    return 1000;
  return std::max(small_level_tpr(M.n_rows, avg), default_tpr(avg));
}
template <typename T>
static void layout_transfer(Ctx* c, const Csr<double>& M, LMat<T>& out, int split16) {
  const int d = transfer_default(M, M.nnz > 0 && M.n_rows >= sell_min_rows() ? sell_stored(c, M) : 0);
  if (d == 1000)
    to_layout<T>(c, M, kFmtSELL, 1, false, out, sell16_enabled() ? split16 : -1);
  else
    to_layout<T>(c, M, kFmtCSR, d, false, out);
}

template <typename T>
static void finalize_levels(Ctx* c, std::vector<BuildLevel<T>>& bl, Union<T>& U, int autotune) {
  const int nl = (int)bl.size();
  int* err = c->err_flag();
  // extended stored order (stored rows, then dense members' rows) and its inverse
  std::vector<DBuf<int>> pext(nl), sinv(nl);
  for (int l = 0; l < nl; ++l) {
    auto& b = bl[l];
    pext[l].alloc(c, (size_t)std::max(b.n, 1));
    sinv[l].alloc(c, (size_t)std::max(b.n, 1));
    copy_d2d(c, pext[l].get(), b.perm.get(), (size_t)b.nS);
    int pos = b.nS;
    for (auto& d : b.dense) {
      hipLaunchKernelGGL(k_iota, dim3(cdiv(d.n, 256)), dim3(256), 0, c->stream, d.n, d.off,
                         pext[l].get() + pos);
      MGD_CHECK_LAUNCH();
      pos += d.n;
    }
    MGD_REQUIRE(pos == b.n, "internal: extended order does not cover the level");
    if (b.n > 0) {
      hipLaunchKernelGGL(k_invert, dim3(cdiv(b.n, 256)), dim3(256), 0, c->stream, b.n,
                         (const int*)pext[l].get(), sinv[l].get(), err);
      MGD_CHECK_LAUNCH();
    }
  }
  c->check_device_errors("extended stored order");
  U.L.clear();
  U.L.resize(nl);
  for (int l = 0; l < nl; ++l) {
    StepScope st("solve-phase build: stored-order level " + std::to_string(l));
    auto& b = bl[l];
    ULevel<T>& lv = U.L[l];
    lv.n = lv.nX = b.n;
    lv.nS = b.nS;
    lv.nC = b.nC;
    lv.nnz_C = b.nnz_C;
    lv.nnz_F = b.A.nnz - b.nnz_C;
    lv.perm = std::move(pext[l]);
    lv.dinv = std::move(b.dinv);
    lv.dgs = std::move(b.dgs);
    lv.cranges = std::move(b.cranges);
    // columns of A in stored order (each member's rows only reference its own rows)
    if (b.A.nnz > 0) {
      hipLaunchKernelGGL(k_remap, dim3(cdiv(b.A.nnz, 256)), dim3(256), 0, c->stream,
                         (long long)b.A.nnz, (const int*)sinv[l].get(), b.n, b.A.ci.get(), err);
      MGD_CHECK_LAUNCH();
    }
    check_index_structure(c, b.A.n_rows, b.nS, b.A.nnz, b.A.rp.get(), b.A.ci.get(),
                          "stored-order level matrix");
    // dense members: offsets in the extended order
    int pos = b.nS;
    for (auto& d : b.dense) {
      lv.dense.push_back({pos, d.n, d.inv});
      lv.dense_max_n = std::max(lv.dense_max_n, d.n);
      lv.dense_entries += (long long)d.n * d.n;
      pos += d.n;
    }
    if (!lv.dense.empty()) {
      lv.dense_dev.alloc(c, lv.dense.size());
      copy_h2d(c, lv.dense_dev.get(), lv.dense.data(), lv.dense.size());
    }
    if (l + 1 < nl && b.n_coarse > 0) {
      auto& nb = bl[l + 1];
      MGD_REQUIRE(nb.n == b.n_coarse && b.nC == b.n_coarse,
                  "internal: coarse level size differs from the C-block");
      lv.nX_next = nb.n;
      lv.nC_next = nb.nC;
      lv.nS_next = nb.nS;
      // W: columns to level l+1 extended order
      if (b.W.nnz > 0) {
        hipLaunchKernelGGL(k_remap, dim3(cdiv(b.W.nnz, 256)), dim3(256), 0, c->stream,
                           (long long)b.W.nnz, (const int*)sinv[l + 1].get(), nb.n, b.W.ci.get(),
                           err);
        MGD_CHECK_LAUNCH();
      }
      // C-block position -> level l+1 index; level l+1 index -> C-block position
      lv.cmap.alloc(c, (size_t)std::max(b.nC, 1));
      lv.cpos.alloc(c, (size_t)std::max(nb.n, 1));
      DBuf<int> cinv;
      if (b.cnat.p) {
        hipLaunchKernelGGL(k_compose, dim3(cdiv(b.nC, 256)), dim3(256), 0, c->stream, b.nC,
                           (const int*)sinv[l + 1].get(), nb.n, (const int*)b.cnat.get(),
                           lv.cmap.get(), err);
        MGD_CHECK_LAUNCH();
        cinv.alloc(c, (size_t)std::max(b.nC, 1));
        hipLaunchKernelGGL(k_invert, dim3(cdiv(b.nC, 256)), dim3(256), 0, c->stream, b.nC,
                           (const int*)b.cnat.get(), cinv.get(), err);
        MGD_CHECK_LAUNCH();
      } else {
        copy_d2d(c, lv.cmap.get(), sinv[l + 1].get(), (size_t)b.nC);
      }
      // rows of W^T in level l+1 extended order
      Csr<double> Wt2;
      Wt2.n_rows = nb.n;
      Wt2.n_cols = b.Wt.n_cols;
      Wt2.nnz = b.Wt.nnz;
      Wt2.rp.alloc(c, (size_t)nb.n + 1);
      Wt2.ci.alloc(c, (size_t)std::max(b.Wt.nnz, 1));
      Wt2.v.alloc(c, (size_t)std::max(b.Wt.nnz, 1));
      {
        // level l+1's extended order is pext[l+1] (moved into U.L[l+1] later)
        const int* src = pext[l + 1].get();
        if (b.cnat.p) {
          hipLaunchKernelGGL(k_compose, dim3(cdiv(nb.n, 256)), dim3(256), 0, c->stream, nb.n,
                             (const int*)cinv.get(), b.nC, src, lv.cpos.get(), err);
          MGD_CHECK_LAUNCH();
        } else {
          copy_d2d(c, lv.cpos.get(), src, (size_t)nb.n);
        }
        DBuf<int> len(c, (size_t)nb.n + 1);
        hipLaunchKernelGGL(k_gather_len, dim3(cdiv(nb.n, 256)), dim3(256), 0, c->stream, nb.n,
                           (const int*)b.Wt.rp.get(), src, len.get());
        MGD_CHECK_LAUNCH();
        const int tot = exclusive_scan_total(c, len.get(), Wt2.rp.get(), nb.n);
        MGD_REQUIRE(tot == b.Wt.nnz, "internal: permuted W^T lost entries");
        hipLaunchKernelGGL(k_gather_rows, dim3(cdiv(nb.n, 256)), dim3(256), 0, c->stream, nb.n,
                           (const int*)b.Wt.rp.get(), (const int*)b.Wt.ci.get(),
                           (const double*)b.Wt.v.get(), src, (const int*)Wt2.rp.get(),
                           Wt2.ci.get(), Wt2.v.get(), err);
        MGD_CHECK_LAUNCH();
      }
      c->check_device_errors("transfer operators in stored order");
      check_index_structure(c, b.W.n_rows, nb.n, b.W.nnz, b.W.rp.get(), b.W.ci.get(),
                            "stored-order interpolation");
      check_index_structure(c, Wt2.n_rows, b.nS - b.nC, Wt2.nnz, Wt2.rp.get(), Wt2.ci.get(),
                            "stored-order restriction");
      // W gathers from three regions of the next level: 32-bit columns;
      // W^T's columns are F indices, one region
      layout_transfer<T>(c, b.W, lv.W, -1);
      tune_restrict<T>(c, lv, b.nS, b.nC, nb.nC, Wt2, lv.Wt, autotune, sizeof(T) == 4);
    }
    c->check_device_errors("stored-order level");
    tune_layout<T>(c, lv, b.A, autotune, sizeof(T) == 4);
  }
  // workspace
  U.B.resize(nl);
  U.X0.resize(nl);
  U.X1.resize(nl);
  U.R.resize(nl);
  U.n0 = nl ? U.L[0].nX : 0;
  for (int l = 0; l < nl; ++l) {
    auto& lv = U.L[l];
    U.B[l].alloc(c, (size_t)std::max(lv.nX, 1));
    U.X0[l].alloc(c, (size_t)std::max(lv.nX, 1));
    U.X1[l].alloc(c, (size_t)std::max(lv.nX, 1));
    U.R[l].alloc(c, (size_t)std::max(lv.nS, 1));
  }
  U.t1.alloc(c, (size_t)std::max(U.n0, 1));
}

// Layout of a level matrix: the tuned choice cached per (rows, nnz, longest
// row) key as code + (threads per workgroup / 64) * kTuneBsUnit, code 1000 =
// SELL, t = CSR with t lanes per row (a value below kTuneBsUnit keeps 256
// threads); without a cached choice and with autotuning off, SELL when
// padding stays within 30%, else CSR with a lane count from the mean row
// length, on 256-thread workgroups.  Autotuning times the residual kernel for
// every layout with 64, 128 and 256 threads per workgroup (rows per workgroup
// = threads / lanes per row; 64-row slices for SELL): the best of three runs
// of back-to-back launches (enough launches for about 0.2 ms per run), and
// keeps the fastest unless the default layout is within kTuneMargin of it, so
// that timing noise does not pick the layout.  A restriction W^T is tuned the
// same way with the restriction kernel (its own cache entries).  Only matrices
// of at least tune_min_rows() rows are timed.
constexpr int kTuneSell = 1000;
constexpr int kTuneBsUnit = 100000;
constexpr double kTuneMargin = 1.03;

static int max_row_len(Ctx* c, int rows, const int* rp) {
  DBuf<int> mr(c, 1);
  fill<int>(c, mr.get(), 0, 1);
  if (rows > 0) {
    hipLaunchKernelGGL(k_max_row, dim3(cdiv(rows, 256)), dim3(256), 0, c->stream, rows, rp,
                       mr.get());
    MGD_CHECK_LAUNCH();
  }
  return read1(c, mr.get());
}
// candidate layouts: SELL while its padding stays within 2x, CSR with 1 lane
// and with up to twice the mean row length in lanes, and the default
static std::vector<int> tune_layouts(long long sell_entries, long long nnz, double avg, int dflt) {
  std::vector<int> layouts;
  if (sell_entries <= 2 * nnz) layouts.push_back(kTuneSell);
  for (int t : {1, 2, 4, 8, 16, 32})
    if (t == 1 || t <= 2 * std::max(avg, 1.0)) layouts.push_back(t);
  if (std::find(layouts.begin(), layouts.end(), dflt) == layouts.end()) layouts.push_back(dflt);
  return layouts;
}
// the timed choice among layouts x {64, 128, 256} threads: apply(value) sets a
// layout up, run() launches the kernel once on it; reps launches per run
template <typename Apply, typename Run>
static int tune_pick(Ctx* c, const std::vector<int>& layouts, int dflt, int reps,
                     const Apply& apply, const Run& run) {
  hipEvent_t e0, e1;
  MGD_HIP(hipEventCreate(&e0));
  MGD_HIP(hipEventCreate(&e1));
  const int dflt_value = dflt + 4 * kTuneBsUnit;  // the default layout, 256 threads
  float best = 1e30f, t_dflt = 1e30f;
  int bt = dflt_value;
  const bool prof = c->profiling;
  c->profiling = false;
  for (int code : layouts)
    for (int bs : {64, 128, 256}) {
      const int cand = code + (bs / 64) * kTuneBsUnit;
      apply(cand);
      run();
      float ms = 1e30f;
      for (int trial = 0; trial < 3; ++trial) {
        MGD_HIP(hipEventRecord(e0, c->stream));
        for (int rep = 0; rep < reps; ++rep) run();
        MGD_HIP(hipEventRecord(e1, c->stream));
        MGD_HIP(hipEventSynchronize(e1));
        float t = 0;
        MGD_HIP(hipEventElapsedTime(&t, e0, e1));
        ms = std::min(ms, t);
      }
      if (cand == dflt_value) t_dflt = ms;
      if (ms < best) {
        best = ms;
        bt = cand;
      }
    }
  if (t_dflt <= best * kTuneMargin) bt = dflt_value;
  c->profiling = prof;
  MGD_HIP(hipEventDestroy(e0));
  MGD_HIP(hipEventDestroy(e1));
  return bt;
}
// launches per timed run: about 0.2 ms of work at 5 TB/s, 4 to 64 launches
static int tune_reps(double bytes) {
  return (int)std::min(64.0, std::max(4.0, 1e9 / std::max(bytes, 1.0)));
}

template <typename T>
static void tune_layout(Ctx* c, ULevel<T>& lv, const Csr<double>& A, int autotune, bool fp32) {
  if (lv.nS == 0) {
    to_layout<T>(c, A, kFmtCSR, 1, true, lv.A);
    return;
  }
  const int maxrow = max_row_len(c, lv.nS, A.rp.get());
  const double avg = (double)A.nnz / lv.nS;
  const long long st = sell_stored(c, A);
  auto apply = [&](int value) {
    const int code = value % kTuneBsUnit, units = value / kTuneBsUnit;
    if (code == kTuneSell)
      to_layout<T>(c, A, kFmtSELL, 1, true, lv.A, sell16_enabled() ? lv.nC : -1);
    else
      to_layout<T>(c, A, kFmtCSR, code, true, lv.A);
    lv.A.bs = units ? 64 * units : 256;
  };
  const int cached = autotune_lookup(lv.nS, A.nnz, maxrow, fp32);
  if (cached > 0) {
    apply(cached);
    return;
  }
  // enough lanes to occupy the device on small levels (a lane per row serialises
  // long rows), SELL when the level is large and its padding small
  const int dflt = (lv.nS >= sell_min_rows() && st <= (long long)(1.3 * A.nnz))
                       ? kTuneSell
                       : std::max(small_level_tpr(lv.nS, avg), default_tpr(avg));
  if (!autotune || lv.nS < tune_min_rows()) {
    apply(dflt);
    return;
  }
  DBuf<T> x(c, (size_t)std::max(lv.nX, 1)), bb(c, (size_t)lv.nS), r(c, (size_t)lv.nS);
  fill<T>(c, x.get(), (T)1, (size_t)std::max(lv.nX, 1));
  fill<T>(c, bb.get(), (T)1, (size_t)lv.nS);
  const auto g = gather_cf<T>(x.get(), x.get(), lv.nC);
  auto run = [&]() {
    ResidL<T> launch{c, lv.A, lv.nS, bb.get(), g, r.get()};
    with_layout(lv.A.fmt, lv.A.tpr, launch);
  };
  const int reps = tune_reps((double)A.nnz * (sizeof(T) + 4) + 4.0 * sizeof(T) * lv.nS);
  const int bt = tune_pick(c, tune_layouts(st, A.nnz, avg, dflt), dflt, reps, apply, run);
  apply(bt);
  autotune_store(lv.nS, A.nnz, maxrow, fp32, bt);
}

// Layout of the restriction W^T of level l (rows: level l+1 in its extended
// order, columns: level l's F-block), chosen like a level matrix's with the
// restriction kernel timed into scratch vectors of the two levels' sizes
// (cpos, the C-block position of each coarse row, is the level's own).
template <typename T>
static void tune_restrict(Ctx* c, const ULevel<T>& lv, int nS, int nC, int nCn,
                          const Csr<double>& Wt, LMat<T>& out, int autotune, bool fp32) {
  if (Wt.n_rows == 0 || Wt.nnz == 0) {
    layout_transfer<T>(c, Wt, out, 0);
    return;
  }
  const int maxrow = max_row_len(c, Wt.n_rows, Wt.rp.get());
  auto apply = [&](int value) {
    const int code = value % kTuneBsUnit, units = value / kTuneBsUnit;
    if (code == kTuneSell)
      to_layout<T>(c, Wt, kFmtSELL, 1, false, out, sell16_enabled() ? 0 : -1);
    else
      to_layout<T>(c, Wt, kFmtCSR, code, false, out);
    out.bs = units ? 64 * units : 256;
  };
  const int cached = autotune_lookup(Wt.n_rows, Wt.nnz, maxrow, fp32, "wt:");
  if (cached > 0) {
    apply(cached);
    return;
  }
  if (!autotune || Wt.n_rows < tune_min_rows()) {
    layout_transfer<T>(c, Wt, out, 0);
    return;
  }
  const double avg = (double)Wt.nnz / Wt.n_rows;
  const long long st = sell_stored(c, Wt);
  const int dflt = transfer_default(Wt, st);
  const int nXn = Wt.n_rows;
  DBuf<T> R(c, (size_t)std::max(nS, 1)), dn(c, (size_t)std::max(nCn, 1));
  DBuf<T> Bn(c, (size_t)nXn), XCn(c, (size_t)std::max(nCn, 1));
  fill<T>(c, R.get(), (T)1, (size_t)std::max(nS, 1));
  fill<T>(c, dn.get(), (T)1, (size_t)std::max(nCn, 1));
  auto run = [&]() {
    RestrictL<T> launch{c, out, nXn, nC, nCn, lv.cpos.get(), R.get(), dn.get(), Bn.get(),
                        XCn.get(), true};
    with_layout(out.fmt, out.tpr, launch);
  };
  const int reps = tune_reps((double)Wt.nnz * (sizeof(T) + 4) + 3.0 * sizeof(T) * nXn);
  const int bt = tune_pick(c, tune_layouts(st, Wt.nnz, avg, dflt), dflt, reps, apply, run);
  apply(bt);
  autotune_store(Wt.n_rows, Wt.nnz, maxrow, fp32, bt, "wt:");
}

template struct Union<double>;
template struct Union<float>;
template std::unique_ptr<Union<double>> build_union<double>(
    Ctx*, const std::vector<const SetupHierarchy*>&, int, int, int, int);
template std::unique_ptr<Union<float>> build_union<float>(
    Ctx*, const std::vector<const SetupHierarchy*>&, int, int, int, int);

}  // namespace mgd
