// Solve-phase structures and kernels: union construction, CF-l1-Jacobi
// half-sweeps, residual, restriction, prolongation, dense coarsest solve,
// and the V(n_pre, n_post) cycle driver.
#include <algorithm>
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

template <typename T>
__global__ void k_dinv(int n, const double* __restrict__ d, const int* __restrict__ srow,
                       T* __restrict__ dinv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dinv[srow[i]] = (T)(1.0 / d[i]);
}

template <typename T>
static void csr_to(Ctx* c, Csr<double>& src, Csr<T>& dst) {
  if constexpr (std::is_same<T, double>::value) {
    dst = std::move(src);
  } else {
    dst.n_rows = src.n_rows;
    dst.n_cols = src.n_cols;
    dst.nnz = src.nnz;
    dst.rp = std::move(src.rp);
    dst.ci = std::move(src.ci);
    dst.v.alloc(c, (size_t)src.nnz);
    cast_copy<T, double>(c, dst.v.get(), src.v.get(), (size_t)src.nnz, KC_VEC);
    c->sync();
    src.v.reset();
  }
}

struct MemberAtLevel {
  const SetupHierarchy* H;
  const SetupLevel* lev;
  int kind;  // 0 coarsening, 1 relaxed last level, 2 dense last level
  int off, n, nc;
};

// Tuning of the stored-matrix row-group width on a built level.
template <typename T>
static int tune_level(Ctx* c, ULevel<T>& lv, int autotune, bool fp32);

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

template <typename T>
std::unique_ptr<Union<T>> build_union(Ctx* c, const std::vector<const SetupHierarchy*>& members,
                                      int n_pre, int n_post, int autotune) {
  auto U = std::make_unique<Union<T>>();
  U->n_pre = n_pre;
  U->n_post = n_post;
  U->members = (int)members.size();
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
    ULevel<T> lv;
    lv.n = off;
    lv.nC = nCtot;
    lv.nS = nCtot + nFtot;
    lv.n_coarse = ncoarse;
    const int nS = lv.nS, nF = nFtot;
    lv.perm.alloc(c, (size_t)std::max(nS, 1));
    lv.dinv.alloc(c, (size_t)std::max(nS, 1));
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
        lv.dense_max_n = std::max(lv.dense_max_n, m.n);
        lv.dense_entries += (long long)m.n * m.n;
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
    // nnz split between the C-block and the F-block (for byte accounting)
    if (nS > 0) {
      int rpC = read1(c, Ad.rp.get() + nCtot);
      lv.nnz_S_C = rpC;
      lv.nnz_S_F = Ad.nnz - rpC;
    }
    csr_to<T>(c, Ad, lv.A);
    csr_to<T>(c, Wd, lv.W);
    if (ncoarse > 0) csr_to<T>(c, Wtd, lv.Wt);
    if (!lv.dense.empty()) {
      lv.dense_dev.alloc(c, lv.dense.size());
      copy_h2d(c, lv.dense_dev.get(), lv.dense.data(), lv.dense.size());
    }
    lv.tpr_w = default_tpr(nF ? (double)lv.W.nnz / nF : 1.0);
    lv.tpr_wt = default_tpr(ncoarse ? (double)lv.Wt.nnz / ncoarse : 1.0);
    U->L.push_back(std::move(lv));
    if (ncoarse == 0) break;
  }
  // workspace
  const size_t nl = U->L.size();
  U->b.resize(nl);
  U->X0.resize(nl);
  U->X1.resize(nl);
  U->r.resize(nl);
  U->n0 = U->L.empty() ? 0 : U->L[0].n;
  for (size_t l = 0; l < nl; ++l) {
    auto& lv = U->L[l];
    if (l > 0) {
      U->b[l].alloc(c, (size_t)std::max(lv.n, 1));
      U->X1[l].alloc(c, (size_t)std::max(lv.n, 1));
    }
    U->X0[l].alloc(c, (size_t)std::max(lv.n, 1));
    U->r[l].alloc(c, (size_t)std::max(lv.nS, 1));
  }
  U->t0.alloc(c, (size_t)std::max(U->n0, 1));
  U->t1.alloc(c, (size_t)std::max(U->n0, 1));
  for (size_t l = 0; l < nl; ++l) {
    StepScope st("solve-phase build: row-group tuning, level " + std::to_string(l));
    U->L[l].tpr = tune_level(c, U->L[l], autotune, sizeof(T) == 4);
  }
  c->sync();
  return U;
}

// ===========================================================================
// solve kernels
// ===========================================================================
template <typename T>
__global__ void k_pre_c(int nS, int nC, const int* __restrict__ perm, const T* __restrict__ dinv,
                        const T* __restrict__ b, T* __restrict__ X) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nS) return;
  const int i = perm[k];
  X[i] = k < nC ? b[i] * dinv[k] : (T)0;
}

template <typename T>
__global__ void k_zero_stored(int nS, const int* __restrict__ perm, T* __restrict__ X) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nS) X[perm[k]] = (T)0;
}

// Xout_S = Xin_S + (b_S - (A Xin)_S) / d_S on stored rows [s0, s1); the
// other stored rows are copied.
template <typename T, int TPR>
__global__ void __launch_bounds__(256) k_half(int nS, int s0, int s1, const int* __restrict__ rp,
                                              const int* __restrict__ ci, const T* __restrict__ v,
                                              const int* __restrict__ perm,
                                              const T* __restrict__ dinv, const T* __restrict__ b,
                                              const T* __restrict__ Xin, T* __restrict__ Xout) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int k = (int)(t / TPR), lane = (int)(t % TPR);
  if (k >= nS) return;
  const int i = perm[k];
  if (k >= s0 && k < s1) {
    const T s = row_dot<TPR, T>(rp, ci, v, Xin, k, lane);
    if (lane == 0) Xout[i] = Xin[i] + (b[i] - s) * dinv[k];
  } else if (lane == 0) {
    Xout[i] = Xin[i];
  }
}

template <typename T, int TPR, bool NATURAL>
__global__ void __launch_bounds__(256) k_resid(int nS, const int* __restrict__ rp,
                                               const int* __restrict__ ci,
                                               const T* __restrict__ v,
                                               const int* __restrict__ perm,
                                               const T* __restrict__ b, const T* __restrict__ X,
                                               T* __restrict__ r) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int k = (int)(t / TPR), lane = (int)(t % TPR);
  if (k >= nS) return;
  const T s = row_dot<TPR, T>(rp, ci, v, X, k, lane);
  if (lane == 0) {
    const int i = perm[k];
    r[NATURAL ? i : k] = b[i] - s;
  }
}

template <typename T, int TPR>
__global__ void __launch_bounds__(256) k_restrict(int nc, int nC, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ v,
                                                  const T* __restrict__ r, T* __restrict__ bc) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int I = (int)(t / TPR), lane = (int)(t % TPR);
  if (I >= nc) return;
  const T s = row_dot<TPR, T>(rp, ci, v, r + nC, I, lane);
  if (lane == 0) bc[I] = r[I] + s;
}

template <typename T, int TPR>
__global__ void __launch_bounds__(256) k_prolong(int nS, int nC, const int* __restrict__ rp,
                                                 const int* __restrict__ ci,
                                                 const T* __restrict__ v,
                                                 const int* __restrict__ perm,
                                                 const T* __restrict__ e, T* __restrict__ X) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int k = (int)(t / TPR), lane = (int)(t % TPR);
  if (k >= nS) return;
  T s;
  if (k < nC) {
    s = e[k];
  } else {
    s = row_dot<TPR, T>(rp, ci, v, e, k - nC, lane);
  }
  if (lane == 0) X[perm[k]] += s;
}

// x = A^{-1} b for every dense-solved member (FP64 arithmetic)
// One workgroup column of 64 rows per member; the loop is unrolled so that
// eight coalesced column loads are in flight per step (the sum stays in
// ascending j).
template <typename T>
__global__ void __launch_bounds__(64) k_dense(const DenseDev* __restrict__ tab,
                                              const T* __restrict__ b, T* __restrict__ X) {
  const DenseDev d = tab[blockIdx.y];
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= d.n) return;
  const double* __restrict__ col = d.inv + i;
  const T* __restrict__ bb = b + d.off;
  double s = 0.0;
  int j = 0;
  for (; j + 8 <= d.n; j += 8) {
    double a[8], x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      a[q] = col[(size_t)(j + q) * d.n];
      x[q] = (double)bb[j + q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) s += a[q] * x[q];
  }
  for (; j < d.n; ++j) s += col[(size_t)j * d.n] * (double)bb[j];
  X[d.off + i] = (T)s;
}

template <typename T>
__global__ void k_axpy_t(int n, const T* __restrict__ x, T* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
struct HalfArgs {
  const ULevel<T>* lv;
  int s0, s1;
  const T *b, *Xin;
  T* Xout;
};
template <int TPR>
struct HalfLaunchD {
  template <typename T>
  static void run(Ctx* c, const HalfArgs<T>& a) {
    const auto& lv = *a.lv;
    const int grid = cdiv((long long)lv.nS * TPR, 256);
    hipLaunchKernelGGL((k_half<T, TPR>), dim3(grid), dim3(256), 0, c->stream, lv.nS, a.s0, a.s1,
                       lv.A.rp.get(), lv.A.ci.get(), lv.A.v.get(), lv.perm.get(), lv.dinv.get(),
                       a.b, a.Xin, a.Xout);
    MGD_CHECK_LAUNCH();
  }
};
template <int TPR>
struct ResidLaunch {
  template <typename T>
  static void run(Ctx* c, const ULevel<T>* lv, const T* b, const T* X, T* r, bool natural) {
    const int grid = cdiv((long long)lv->nS * TPR, 256);
    if (natural)
      hipLaunchKernelGGL((k_resid<T, TPR, true>), dim3(grid), dim3(256), 0, c->stream, lv->nS,
                         lv->A.rp.get(), lv->A.ci.get(), lv->A.v.get(), lv->perm.get(), b, X, r);
    else
      hipLaunchKernelGGL((k_resid<T, TPR, false>), dim3(grid), dim3(256), 0, c->stream, lv->nS,
                         lv->A.rp.get(), lv->A.ci.get(), lv->A.v.get(), lv->perm.get(), b, X, r);
    MGD_CHECK_LAUNCH();
  }
};
template <int TPR>
struct RestrictLaunch {
  template <typename T>
  static void run(Ctx* c, const ULevel<T>* lv, const T* r, T* bc) {
    const int grid = cdiv((long long)lv->n_coarse * TPR, 256);
    hipLaunchKernelGGL((k_restrict<T, TPR>), dim3(grid), dim3(256), 0, c->stream, lv->n_coarse,
                       lv->nC, lv->Wt.rp.get(), lv->Wt.ci.get(), lv->Wt.v.get(), r, bc);
    MGD_CHECK_LAUNCH();
  }
};
template <int TPR>
struct ProlongLaunch {
  template <typename T>
  static void run(Ctx* c, const ULevel<T>* lv, const T* e, T* X) {
    const int grid = cdiv((long long)lv->nS * TPR, 256);
    hipLaunchKernelGGL((k_prolong<T, TPR>), dim3(grid), dim3(256), 0, c->stream, lv->nS, lv->nC,
                       lv->W.rp.get(), lv->W.ci.get(), lv->W.v.get(), lv->perm.get(), e, X);
    MGD_CHECK_LAUNCH();
  }
};

template <template <int> class K, typename... Args>
static void dispatch(int tpr, Args&&... args) {
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

// algorithmic bytes (each entry/index/vector element once per launch)
template <typename T>
static double half_bytes(const ULevel<T>& lv, bool c_half) {
  const double ts = sizeof(T);
  const long long rows = c_half ? lv.nC : lv.nS - lv.nC;
  const long long nnz = c_half ? lv.nnz_S_C : lv.nnz_S_F;
  return nnz * (ts + 4) + rows * (4 + 2 * ts) + lv.nS * (4 + 2 * ts) + (double)lv.n * 0;
}
template <typename T>
static double resid_bytes(const ULevel<T>& lv) {
  const double ts = sizeof(T);
  return (double)lv.A.nnz * (ts + 4) + lv.nS * (4 + 4 + 2 * ts) + (double)lv.n * ts;
}

static inline int cls_of(int l, int cls0) { return l == 0 ? cls0 : KC_VCYCLE_COARSE; }
template <typename T>
static std::string khalf(const Ctx* c, int tpr) {
  return ksym(c, "k_half", {type_name<T>(), std::to_string(tpr_of(tpr))});
}
template <typename T>
static std::string kresid(const Ctx* c, int tpr, bool natural) {
  return ksym(c, "k_resid", {type_name<T>(), std::to_string(tpr_of(tpr)), natural ? "true" : "false"});
}

template <typename T>
void Union<T>::vcycle(Ctx* c, const T* b0, T* x0) {
  const int nl = (int)L.size();
  auto Bp = [&](int l) -> const T* { return l == 0 ? b0 : b[l].get(); };
  auto X1p = [&](int l) -> T* { return l == 0 ? x0 : X1[l].get(); };
  for (int l = 0; l < nl; ++l) {
    ULevel<T>& lv = L[l];
    T* x1 = X1p(l);
    T* xw = X0[l].get();
    const T* bl = Bp(l);
    if (lv.nS > 0) {
      if (n_pre == 0) {
        hipLaunchKernelGGL(k_zero_stored<T>, dim3(cdiv(lv.nS, 256)), dim3(256), 0, c->stream,
                           lv.nS, lv.perm.get(), x1);
        MGD_CHECK_LAUNCH();
      }
      for (int s = 0; s < n_pre; ++s) {
        if (s == 0) {
          ProfScope ps(c, cls_of(l, KC_SMOOTH_L0),
                       (double)lv.nS * (4 + 2 * sizeof(T)) + lv.nC * (sizeof(T)),
                       ksym(c, "k_pre_c", {type_name<T>()}));
          hipLaunchKernelGGL(k_pre_c<T>, dim3(cdiv(lv.nS, 256)), dim3(256), 0, c->stream, lv.nS,
                             lv.nC, lv.perm.get(), lv.dinv.get(), bl, xw);
          MGD_CHECK_LAUNCH();
        } else {
          ProfScope ps(c, cls_of(l, KC_SMOOTH_L0), half_bytes(lv, true), khalf<T>(c, lv.tpr));
          dispatch<HalfLaunchD>(lv.tpr, c, HalfArgs<T>{&lv, 0, lv.nC, bl, x1, xw});
        }
        ProfScope ps(c, cls_of(l, KC_SMOOTH_L0), half_bytes(lv, false), khalf<T>(c, lv.tpr));
        dispatch<HalfLaunchD>(lv.tpr, c, HalfArgs<T>{&lv, lv.nC, lv.nS, bl, xw, x1});
      }
      if (lv.n_coarse > 0) {
        {
          ProfScope ps(c, cls_of(l, KC_RESID_L0), resid_bytes(lv), kresid<T>(c, lv.tpr, false));
          dispatch<ResidLaunch>(lv.tpr, c, &lv, bl, (const T*)x1, r[l].get(), false);
        }
        ProfScope ps(c, cls_of(l, KC_TRANSFER_L0),
                     (double)lv.Wt.nnz * (sizeof(T) + 4) + lv.n_coarse * (4 + sizeof(T)) +
                         (double)lv.nS * sizeof(T),
                     ksym(c, "k_restrict", {type_name<T>(), std::to_string(tpr_of(lv.tpr_wt))}));
        dispatch<RestrictLaunch>(lv.tpr_wt, c, &lv, (const T*)r[l].get(), b[l + 1].get());
      }
    }
    if (!lv.dense.empty()) {
      ProfScope ps(c, KC_COARSE_SOLVE, 8.0 * lv.dense_entries + 2.0 * sizeof(T) * lv.n,
                   ksym(c, "k_dense", {type_name<T>()}));
      dim3 grid(cdiv(lv.dense_max_n, 64), (unsigned)lv.dense.size());
      hipLaunchKernelGGL(k_dense<T>, grid, dim3(64), 0, c->stream,
                         (const DenseDev*)lv.dense_dev.get(), bl, x1);
      MGD_CHECK_LAUNCH();
    }
  }
  for (int l = nl - 1; l >= 0; --l) {
    ULevel<T>& lv = L[l];
    if (lv.nS == 0) continue;
    T* x1 = X1p(l);
    T* xw = X0[l].get();
    const T* bl = Bp(l);
    if (lv.n_coarse > 0) {
      ProfScope ps(c, cls_of(l, KC_TRANSFER_L0),
                   (double)lv.W.nnz * (sizeof(T) + 4) + lv.nS * (4 + 2.0 * sizeof(T)) +
                       lv.n_coarse * (double)sizeof(T),
                   ksym(c, "k_prolong", {type_name<T>(), std::to_string(tpr_of(lv.tpr_w))}));
      dispatch<ProlongLaunch>(lv.tpr_w, c, &lv, (const T*)X1p(l + 1), x1);
    }
    for (int s = 0; s < n_post; ++s) {
      {
        ProfScope ps(c, cls_of(l, KC_SMOOTH_L0), half_bytes(lv, false), khalf<T>(c, lv.tpr));
        dispatch<HalfLaunchD>(lv.tpr, c, HalfArgs<T>{&lv, lv.nC, lv.nS, bl, x1, xw});
      }
      ProfScope ps(c, cls_of(l, KC_SMOOTH_L0), half_bytes(lv, true), khalf<T>(c, lv.tpr));
      dispatch<HalfLaunchD>(lv.tpr, c, HalfArgs<T>{&lv, 0, lv.nC, bl, xw, x1});
    }
  }
}

template <typename T>
void Union<T>::apply(Ctx* c, const T* bvec, T* z, int cycles) {
  vcycle(c, bvec, z);
  for (int k = 1; k < cycles; ++k) {
    ULevel<T>& lv = L[0];
    if (!lv.dense.empty()) fill<T>(c, t0.get(), (T)0, (size_t)n0);
    if (lv.nS > 0) {
      ProfScope ps(c, KC_RESID_L0, resid_bytes(lv), kresid<T>(c, lv.tpr, true));
      dispatch<ResidLaunch>(lv.tpr, c, &lv, bvec, (const T*)z, t0.get(), true);
    }
    vcycle(c, t0.get(), t1.get());
    hipLaunchKernelGGL(k_axpy_t<T>, dim3(cdiv(n0, 256)), dim3(256), 0, c->stream, n0,
                       (const T*)t1.get(), z);
    MGD_CHECK_LAUNCH();
  }
}

template <typename T>
double Union<T>::bytes_per_vcycle() const {
  double s = 0;
  for (auto& lv : L) {
    if (lv.nS > 0) {
      s += (double)lv.nS * (4 + 2 * sizeof(T)) + lv.nC * sizeof(T);
      s += half_bytes(lv, false) * (n_pre + n_post) + half_bytes(lv, true) * (n_pre + n_post - 1);
      if (lv.n_coarse > 0) {
        s += resid_bytes(lv);
        s += (double)lv.Wt.nnz * (sizeof(T) + 4) + lv.n_coarse * (4 + sizeof(T)) +
             (double)lv.nS * sizeof(T);
        s += (double)lv.W.nnz * (sizeof(T) + 4) + lv.nS * (4 + 2.0 * sizeof(T)) +
             lv.n_coarse * (double)sizeof(T);
      }
    }
    s += 8.0 * lv.dense_entries;
  }
  return s;
}

// ===========================================================================
// autotuning of row-group widths
// ===========================================================================
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune;
static bool g_tune_loaded = false;

static std::string tune_key(long long rows, long long nnz, int maxrow, bool fp32) {
  std::ostringstream o;
  o << (fp32 ? "f32:" : "f64:") << rows << ":" << nnz << ":" << maxrow;
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
int autotune_lookup(long long rows, long long nnz, int maxrow, bool fp32) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(tune_key(rows, nnz, maxrow, fp32));
  return it == g_tune.end() ? 0 : it->second;
}
void autotune_store(long long rows, long long nnz, int maxrow, bool fp32, int tpr) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  tune_load_locked();
  g_tune[tune_key(rows, nnz, maxrow, fp32)] = tpr;
  tune_save_locked();
}

__global__ void k_max_row(int n, const int* __restrict__ rp, int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int m = i < n ? rp[i + 1] - rp[i] : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(out, m);
}

template <typename T>
static int tune_level(Ctx* c, ULevel<T>& lv, int autotune, bool fp32) {
  if (lv.nS == 0) return 1;
  DBuf<int> mr(c, 1);
  fill<int>(c, mr.get(), 0, 1);
  hipLaunchKernelGGL(k_max_row, dim3(cdiv(lv.nS, 256)), dim3(256), 0, c->stream, lv.nS,
                     lv.A.rp.get(), mr.get());
  MGD_CHECK_LAUNCH();
  const int maxrow = read1(c, mr.get());
  const double avg = (double)lv.A.nnz / lv.nS;
  int t = autotune_lookup(lv.nS, lv.A.nnz, maxrow, fp32);
  if (t > 0) return t;
  if (!autotune) return default_tpr(avg);
  DBuf<T> x(c, (size_t)lv.n), y(c, (size_t)lv.nS);
  fill<T>(c, x.get(), (T)1, (size_t)lv.n);
  hipEvent_t e0, e1;
  MGD_HIP(hipEventCreate(&e0));
  MGD_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bt = default_tpr(avg);
  const bool prof = c->profiling;
  c->profiling = false;
  for (int cand : {1, 2, 4, 8, 16, 32}) {
    if (cand > 1 && cand > 2 * std::max(avg, 1.0)) break;
    dispatch<ResidLaunch>(cand, c, (const ULevel<T>*)&lv, (const T*)x.get(), (const T*)x.get(),
                          y.get(), false);
    MGD_HIP(hipEventRecord(e0, c->stream));
    for (int rep = 0; rep < 5; ++rep)
      dispatch<ResidLaunch>(cand, c, (const ULevel<T>*)&lv, (const T*)x.get(), (const T*)x.get(),
                            y.get(), false);
    MGD_HIP(hipEventRecord(e1, c->stream));
    MGD_HIP(hipEventSynchronize(e1));
    float ms = 0;
    MGD_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      bt = cand;
    }
  }
  c->profiling = prof;
  MGD_HIP(hipEventDestroy(e0));
  MGD_HIP(hipEventDestroy(e1));
  autotune_store(lv.nS, lv.A.nnz, maxrow, fp32, bt);
  return bt;
}

template struct Union<double>;
template struct Union<float>;
template std::unique_ptr<Union<double>> build_union<double>(Ctx*,
                                                            const std::vector<const SetupHierarchy*>&,
                                                            int, int, int);
template std::unique_ptr<Union<float>> build_union<float>(Ctx*,
                                                          const std::vector<const SetupHierarchy*>&,
                                                          int, int, int);

}  // namespace mgd
