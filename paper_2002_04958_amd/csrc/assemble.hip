// Assembly of eq. 2.2 from per-cell coefficients, the transposed block
// system, and the adjoint gradient gather.
//
// Assembly follows a fixed evaluation order so that it reproduces a plain
// reference bit for bit: face weight (2 k_c) k_nb / (k_c + k_nb), optional
// factor (1 + 0.5 xi); diagonal = 0 + faces in direction order -x, +x, -y,
// +y, -z, +z, then the row's coupling magnitudes (E rows: groups ascending,
// then c_EI), then the mass.  No contraction into fused multiply-adds.
#pragma clang fp contract(off)

#include <map>
#include <mutex>

#include "handles.hpp"
#include "kernels.hpp"
#include "spmv.hpp"

using namespace mgd;

namespace {

// Half storage of symmetric blocks for the block matvec (BlockSysDev::sym_*).
struct SymHalf {
  DBuf<int> urp, src;
  long long unnz = 0;
  std::vector<DBuf<double>> uv;
};

struct OwnedSystem {
  std::vector<mgd_csr> desc;
  std::vector<Csr<double>> blocks;   // when blocks have their own patterns
  DBuf<int> rp, ci;                  // shared pattern (assembly)
  std::vector<DBuf<double>> vals;    // per-block values (assembly)
  DBuf<double> d_gE, d_Eg, d_EI, d_IE;
  std::unique_ptr<SymHalf> sym;      // set when every block is symmetric
};

std::mutex g_sys_mu;
std::map<const mgd_csr*, std::unique_ptr<OwnedSystem>> g_systems;

__device__ __forceinline__ int nbr(int c, int d, int n, int dim) {
  const int ix = c % n, iy = (c / n) % n, iz = dim == 3 ? c / (n * n) : 0;
  switch (d) {
    case 0: return ix > 0 ? c - 1 : -1;
    case 1: return ix < n - 1 ? c + 1 : -1;
    case 2: return iy > 0 ? c - n : -1;
    case 3: return iy < n - 1 ? c + n : -1;
    case 4: return iz > 0 ? c - n * n : -1;
    default: return iz < n - 1 ? c + n * n : -1;
  }
}

__global__ void k_pattern_len(int N, int n, int dim, int* __restrict__ len) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  int k = 1;
  for (int d = 0; d < 2 * dim; ++d) k += nbr(c, d, n, dim) >= 0;
  len[c] = k;
}

// sorted columns: -z, -y, -x, c, +x, +y, +z
__global__ void k_pattern_fill(int N, int n, int dim, const int* __restrict__ rp,
                               int* __restrict__ ci, int* __restrict__ err) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  int p = rp[c];
  int len = 1;  // the diagonal plus the interior faces
  for (int d = 0; d < 2 * dim; ++d) len += nbr(c, d, n, dim) >= 0 ? 1 : 0;
  if (rp[c + 1] - p != len) {
    atomicOr(err, 1);
    return;
  }
  const int order[7] = {4, 2, 0, -1, 1, 3, 5};
  for (int q = 0; q < 7; ++q) {
    const int d = order[q];
    if (d < 0) {
      ci[p++] = c;
      continue;
    }
    if (d >= 2 * dim) continue;
    const int j = nbr(c, d, n, dim);
    if (j >= 0) ci[p++] = j;
  }
}

__global__ void k_assemble_values(int G, int N, int n, int dim, const double* __restrict__ kappa,
                                  const double* __restrict__ c_gE, const double* __restrict__ c_Eg,
                                  const double* __restrict__ c_EI, double mass,
                                  const double* __restrict__ xi, const int* __restrict__ rp,
                                  const int* __restrict__ ci, double* const* __restrict__ vals) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (c >= N) return;
  const double* k = kappa + (size_t)a * N;
  double* v = vals[a];
  const int e0 = rp[c], e1 = rp[c + 1];
  double diag = 0.0;
  for (int d = 0; d < 2 * dim; ++d) {
    const int j = nbr(c, d, n, dim);
    if (j < 0) continue;
    const double ka = k[c], kb = k[j];
    double w = (2.0 * ka) * kb / (ka + kb);
    if (xi) w = w * (1.0 + 0.5 * xi[((size_t)a * N + c) * (2 * dim) + d]);
    diag = diag + w;
    for (int e = e0; e < e1; ++e)
      if (ci[e] == j) v[e] = -w;
  }
  if (a < G) {
    diag = diag + c_gE[(size_t)a * N + c];
  } else if (a == G) {
    for (int g = 0; g < G; ++g) diag = diag + c_Eg[(size_t)g * N + c];
    diag = diag + c_EI[c];
  } else {
    diag = diag + c_EI[c];
  }
  diag = diag + mass;
  for (int e = e0; e < e1; ++e)
    if (ci[e] == c) v[e] = diag;
}

__global__ void k_negate(size_t n, const double* __restrict__ a, double* __restrict__ b) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    b[i] = -a[i];
}

__global__ void k_grad_kappa(int G, int N, int n, int dim, const double* __restrict__ kappa,
                             const double* __restrict__ x, const double* __restrict__ lam,
                             double* __restrict__ dk) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (c >= N) return;
  const size_t o = (size_t)a * N;
  const double* k = kappa + o;
  double acc = 0.0;
  for (int d = 0; d < 2 * dim; ++d) {
    const int j = nbr(c, d, n, dim);
    if (j < 0) continue;
    const double dT = -(lam[o + c] - lam[o + j]) * (x[o + c] - x[o + j]);
    const double s = k[c] + k[j];
    acc = acc + dT * (2.0 * k[j] * k[j]) / (s * s);
  }
  dk[o + c] = acc;
}

__global__ void k_grad_coupling(int G, int N, const double* __restrict__ x,
                                const double* __restrict__ lam, double* __restrict__ dc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const size_t E = (size_t)G * N, I = (size_t)(G + 1) * N;
  for (int g = 0; g < G; ++g) {
    const size_t o = (size_t)g * N;
    dc[o + c] = -lam[o + c] * (x[o + c] - x[E + c]);
    dc[(size_t)G * N + o + c] = -lam[E + c] * (x[E + c] - x[o + c]);
  }
  dc[(size_t)2 * G * N + c] = -lam[E + c] * (x[E + c] - x[I + c]) - lam[I + c] * (x[I + c] - x[E + c]);
}

// Per row of a sorted pattern: the diagonal's position and the number of
// entries from it to the row's end; flags[0] = 1 when a row has no diagonal,
// more than kSymMaxRow entries or more than kSymMaxUpper from the diagonal on
// (no half storage then).
__global__ void k_sym_rows(int N, const int* __restrict__ rp, const int* __restrict__ ci,
                           int* __restrict__ dpos, int* __restrict__ ulen,
                           int* __restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int e0 = rp[i], e1 = rp[i + 1];
  int k = e0;
  while (k < e1 && ci[k] < i) ++k;
  if (k == e1 || ci[k] != i || e1 - e0 > kSymMaxRow || e1 - k > kSymMaxUpper) {
    atomicOr(flags, 1);
    dpos[i] = e0;
    ulen[i] = 0;
    return;
  }
  dpos[i] = k;
  ulen[i] = e1 - k;
}

// src[k] for every entry of row i: its own half-storage position on and
// above the diagonal, below it the position of its mirror (j, i), found by
// bisection among row j's entries right of j's diagonal.  flags[0] = 1 when a
// mirror is missing or some block's value differs from its mirror's in any bit.
__global__ void k_sym_src(int N, int nb, const int* __restrict__ rp, const int* __restrict__ ci,
                          const int* __restrict__ dpos, const int* __restrict__ urp,
                          const double* const* __restrict__ vals, int* __restrict__ src,
                          int* __restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int e1 = rp[i + 1];
  for (int k = rp[i]; k < e1; ++k) {
    const int j = ci[k];
    if (j >= i) {
      src[k] = urp[i] + (k - dpos[i]);
      continue;
    }
    int lo = dpos[j] + 1, hi = rp[j + 1] - 1, kj = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int cm = ci[mid];
      if (cm == i) {
        kj = mid;
        break;
      }
      if (cm < i)
        lo = mid + 1;
      else
        hi = mid - 1;
    }
    if (kj < 0) {
      atomicOr(flags, 1);
      src[k] = urp[i];  // a valid position; the half storage is not used
      continue;
    }
    src[k] = urp[j] + (kj - dpos[j]);
    for (int a = 0; a < nb; ++a)
      if (__double_as_longlong(vals[a][k]) != __double_as_longlong(vals[a][kj])) {
        atomicOr(flags, 1);
        break;
      }
  }
}

// block blockIdx.y's values on and above the diagonal, row after row
__global__ void k_sym_fill(int N, const int* __restrict__ rp, const int* __restrict__ dpos,
                           const int* __restrict__ urp, const double* const* __restrict__ vals,
                           double* const* __restrict__ uv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double* __restrict__ v = vals[blockIdx.y];
  double* __restrict__ u = uv[blockIdx.y];
  const int d = dpos[i], e1 = rp[i + 1], o = urp[i];
  for (int k = d; k < e1; ++k) u[o + (k - d)] = v[k];
}

// The half storage of nb blocks sharing the pattern (rp, ci): null when a
// block differs from its transpose in any bit or a row is longer than
// kSymMaxRow.
std::unique_ptr<SymHalf> build_sym(Ctx* c, int N, long long nnz, const int* rp, const int* ci,
                                   const std::vector<const double*>& vals) {
  const int nb = (int)vals.size();
  if (N <= 0 || nnz <= 0 || nb <= 0) return nullptr;
  DBuf<int> dpos(c, (size_t)N), ulen(c, (size_t)N), flags(c, 1);
  fill<int>(c, flags.get(), 0, 1);
  hipLaunchKernelGGL(k_sym_rows, dim3(cdiv(N, 256)), dim3(256), 0, c->stream, N, rp, ci, dpos.get(),
                     ulen.get(), flags.get());
  MGD_CHECK_LAUNCH();
  if (read1(c, flags.get())) return nullptr;
  auto h = std::make_unique<SymHalf>();
  h->urp.alloc(c, (size_t)N + 1);
  h->unnz = exclusive_scan_total(c, ulen.get(), h->urp.get(), N);
  h->src.alloc(c, (size_t)nnz);
  DBuf<const double*> vtab(c, (size_t)nb);
  copy_h2d(c, vtab.get(), vals.data(), (size_t)nb);
  hipLaunchKernelGGL(k_sym_src, dim3(cdiv(N, 256)), dim3(256), 0, c->stream, N, nb, rp, ci,
                     (const int*)dpos.get(), (const int*)h->urp.get(),
                     (const double* const*)vtab.get(), h->src.get(), flags.get());
  MGD_CHECK_LAUNCH();
  if (read1(c, flags.get())) return nullptr;
  std::vector<double*> up(nb);
  h->uv.resize(nb);
  for (int a = 0; a < nb; ++a) {
    h->uv[a].alloc(c, (size_t)std::max(h->unnz, 1LL));
    up[a] = h->uv[a].get();
  }
  DBuf<double*> utab(c, (size_t)nb);
  copy_h2d(c, utab.get(), up.data(), (size_t)nb);
  hipLaunchKernelGGL(k_sym_fill, dim3(cdiv(N, 256), nb), dim3(256), 0, c->stream, N, rp,
                     (const int*)dpos.get(), (const int*)h->urp.get(),
                     (const double* const*)vtab.get(), (double* const*)utab.get());
  MGD_CHECK_LAUNCH();
  c->sync();
  return h;
}

}  // namespace

namespace mgd {
void attach_half_storage(const mgd_block_system* A, BlockSysDev& S) {
  const char* e = std::getenv("MGD_SYM_MATVEC");
  if (e && e[0] == '0') return;
  std::lock_guard<std::mutex> g(g_sys_mu);
  auto it = g_systems.find(A->blocks);
  if (it == g_systems.end() || !it->second->sym) return;
  const SymHalf& h = *it->second->sym;
  if ((int)h.uv.size() != A->G + 2) return;
  S.sym = 1;
  S.sym_urp = h.urp.get();
  S.sym_src = h.src.get();
  S.sym_nnz = h.unnz;
  for (int a = 0; a < A->G + 2; ++a) S.sym_v[a] = h.uv[a].get();
}
}  // namespace mgd

void check_coeffs(const mgd_coeffs* cf) {
  MGD_REQUIRE(cf, "coeffs is NULL");
  MGD_REQUIRE(cf->dim == 2 || cf->dim == 3, "dim must be 2 or 3");
  MGD_REQUIRE(cf->n >= 1 && cf->G >= 1 && cf->G + 2 <= kMaxBlocks, "bad n or G");
  MGD_REQUIRE(cf->kappa && cf->c_gE && cf->c_Eg && cf->c_EI, "coefficient pointer is NULL");
  const long long N = cf->dim == 2 ? (long long)cf->n * cf->n : (long long)cf->n * cf->n * cf->n;
  MGD_REQUIRE((cf->G + 2) * N < INT32_MAX, "system too large for int32 indices");
}

void assemble_impl(Ctx* c, const mgd_coeffs* cf, mgd_block_system* out) {
  check_coeffs(cf);
  const int G = cf->G, n = cf->n, dim = cf->dim;
  const int N = dim == 2 ? n * n : n * n * n;
  auto os = std::make_unique<OwnedSystem>();
  DBuf<int> len(c, (size_t)N);
  hipLaunchKernelGGL(k_pattern_len, dim3(cdiv(N, 256)), dim3(256), 0, c->stream, N, n, dim, len.get());
  MGD_CHECK_LAUNCH();
  os->rp.alloc(c, (size_t)N + 1);
  const int nnz = exclusive_scan_total(c, len.get(), os->rp.get(), N);
  os->ci.alloc(c, (size_t)nnz);
  hipLaunchKernelGGL(k_pattern_fill, dim3(cdiv(N, 256)), dim3(256), 0, c->stream, N, n, dim,
                     (const int*)os->rp.get(), os->ci.get(), c->err_flag());
  MGD_CHECK_LAUNCH();
  c->check_device_errors("stencil pattern fill");
  {
    Csr<double> pat;  // structure check of the shared stencil pattern
    pat.n_rows = pat.n_cols = N;
    pat.nnz = nnz;
    pat.rp = std::move(os->rp);
    pat.ci = std::move(os->ci);
    check_structure(c, pat, "assembled stencil pattern", true);
    os->rp = std::move(pat.rp);
    os->ci = std::move(pat.ci);
  }
  std::vector<double*> vp(G + 2);
  os->vals.resize(G + 2);
  for (int a = 0; a < G + 2; ++a) {
    os->vals[a].alloc(c, (size_t)nnz);
    vp[a] = os->vals[a].get();
  }
  DBuf<double*> vtab(c, (size_t)G + 2);
  copy_h2d(c, vtab.get(), vp.data(), (size_t)G + 2);
  hipLaunchKernelGGL(k_assemble_values, dim3(cdiv(N, 256), G + 2), dim3(256), 0, c->stream, G, N, n,
                     dim, cf->kappa, cf->c_gE, cf->c_Eg, cf->c_EI, cf->mass, cf->xi,
                     (const int*)os->rp.get(), (const int*)os->ci.get(),
                     (double* const*)vtab.get());
  MGD_CHECK_LAUNCH();
  os->d_gE.alloc(c, (size_t)G * N);
  os->d_Eg.alloc(c, (size_t)G * N);
  os->d_EI.alloc(c, (size_t)N);
  os->d_IE.alloc(c, (size_t)N);
  const int gg = std::min(cdiv((long long)G * N, 256), 65535);
  hipLaunchKernelGGL(k_negate, dim3(gg), dim3(256), 0, c->stream, (size_t)G * N, cf->c_gE, os->d_gE.get());
  hipLaunchKernelGGL(k_negate, dim3(gg), dim3(256), 0, c->stream, (size_t)G * N, cf->c_Eg, os->d_Eg.get());
  hipLaunchKernelGGL(k_negate, dim3(cdiv(N, 256)), dim3(256), 0, c->stream, (size_t)N, cf->c_EI, os->d_EI.get());
  hipLaunchKernelGGL(k_negate, dim3(cdiv(N, 256)), dim3(256), 0, c->stream, (size_t)N, cf->c_EI, os->d_IE.get());
  MGD_CHECK_LAUNCH();
  c->sync();
  {
    std::vector<const double*> cv(vp.begin(), vp.end());
    os->sym = build_sym(c, N, nnz, os->rp.get(), os->ci.get(), cv);
  }
  os->desc.resize(G + 2);
  for (int a = 0; a < G + 2; ++a)
    os->desc[a] = {N, N, nnz, os->rp.get(), os->ci.get(), os->vals[a].get()};
  out->G = G;
  out->N = N;
  out->blocks = os->desc.data();
  out->d_gE = os->d_gE.get();
  out->d_Eg = os->d_Eg.get();
  out->d_EI = os->d_EI.get();
  out->d_IE = os->d_IE.get();
  std::lock_guard<std::mutex> g(g_sys_mu);
  g_systems[os->desc.data()] = std::move(os);
}

void system_transpose_impl(Ctx* c, const mgd_block_system* A, mgd_block_system* out) {
  const int G = A->G, N = A->N;
  auto os = std::make_unique<OwnedSystem>();
  os->blocks.resize(G + 2);
  for (int a = 0; a < G + 2; ++a) {
    Csr<double> tmp;
    csr_copy_from(c, &A->blocks[a], tmp);
    transpose(c, tmp, os->blocks[a]);
  }
  os->d_gE.alloc(c, (size_t)G * N);
  os->d_Eg.alloc(c, (size_t)G * N);
  os->d_EI.alloc(c, (size_t)N);
  os->d_IE.alloc(c, (size_t)N);
  copy_d2d(c, os->d_gE.get(), A->d_Eg, (size_t)G * N);
  copy_d2d(c, os->d_Eg.get(), A->d_gE, (size_t)G * N);
  copy_d2d(c, os->d_EI.get(), A->d_IE, (size_t)N);
  copy_d2d(c, os->d_IE.get(), A->d_EI, (size_t)N);
  c->sync();
  // Blocks that share one pattern keep sharing it: the transposes of equal
  // patterns are equal (every transposed row is sorted by column), so block
  // 0's row pointers and column indices serve all blocks.
  bool shared = true;
  for (int a = 1; a < G + 2; ++a)
    shared = shared && A->blocks[a].row_ptr == A->blocks[0].row_ptr &&
             A->blocks[a].col_idx == A->blocks[0].col_idx && A->blocks[a].nnz == A->blocks[0].nnz;
  os->desc.resize(G + 2);
  for (int a = 0; a < G + 2; ++a) {
    auto& B = os->blocks[a];
    if (shared && a > 0) {
      B.rp.reset();
      B.ci.reset();
    }
    const auto& P = shared ? os->blocks[0] : B;
    os->desc[a] = {B.n_rows, B.n_cols, B.nnz, P.rp.get(), P.ci.get(), B.v.get()};
  }
  if (shared) {
    std::vector<const double*> cv(G + 2);
    for (int a = 0; a < G + 2; ++a) cv[a] = os->blocks[a].v.get();
    os->sym = build_sym(c, N, os->blocks[0].nnz, os->blocks[0].rp.get(), os->blocks[0].ci.get(),
                        cv);
  }
  out->G = G;
  out->N = N;
  out->blocks = os->desc.data();
  out->d_gE = os->d_gE.get();
  out->d_Eg = os->d_Eg.get();
  out->d_EI = os->d_EI.get();
  out->d_IE = os->d_IE.get();
  std::lock_guard<std::mutex> g(g_sys_mu);
  g_systems[os->desc.data()] = std::move(os);
}

void system_free_impl(mgd_block_system* s) {
  std::lock_guard<std::mutex> g(g_sys_mu);
  auto it = g_systems.find(s->blocks);
  MGD_REQUIRE(it != g_systems.end(), "block system is not owned by the library");
  g_systems.erase(it);
  s->blocks = nullptr;
}

void adjoint_gradients_impl(Ctx* c, const mgd_coeffs* cf, const double* x, const double* lam,
                            double* dk, double* dc) {
  check_coeffs(cf);
  MGD_REQUIRE(cf->xi == nullptr, "gradients are defined for the symmetric assembly (xi == NULL)");
  const int G = cf->G, n = cf->n, dim = cf->dim;
  const int N = dim == 2 ? n * n : n * n * n;
  if (dk) {
    ProfScope ps(c, KC_VEC, 8.0 * 4 * (G + 2) * N);
    hipLaunchKernelGGL(k_grad_kappa, dim3(cdiv(N, 256), G + 2), dim3(256), 0, c->stream, G, N, n,
                       dim, cf->kappa, x, lam, dk);
    MGD_CHECK_LAUNCH();
  }
  if (dc) {
    hipLaunchKernelGGL(k_grad_coupling, dim3(cdiv(N, 256)), dim3(256), 0, c->stream, G, N, x, lam, dc);
    MGD_CHECK_LAUNCH();
  }
}
