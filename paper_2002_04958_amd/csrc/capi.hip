#include <algorithm>
// The C ABI of libmgdamg: argument checks, context handling and conversion
// of internal errors into status codes.  No exception crosses this file.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "handles.hpp"
#include "kernels.hpp"
#include "rowdot.hpp"

using namespace mgd;

// implemented in other translation units
block_precond* block_precond_create_impl(Ctx* c, const mgd_block_system* A, const block_params* p);
void block_precond_apply_dispatch(block_precond* bp, const double* r, double* z);
mgd_status gmres_impl(Ctx* c, const BlockSysDev& S, block_precond* M, const double* b, double* x,
                      const gmres_params& p, gmres_result& res);
void assemble_impl(Ctx* c, const mgd_coeffs* cf, mgd_block_system* out);
void system_transpose_impl(Ctx* c, const mgd_block_system* A, mgd_block_system* out);
void system_free_impl(mgd_block_system* s);
void adjoint_gradients_impl(Ctx* c, const mgd_coeffs* cf, const double* x, const double* lam,
                            double* dk, double* dc);
void check_coeffs(const mgd_coeffs* cf);

namespace {
thread_local std::string g_last_error;

template <typename F>
mgd_status guard(F&& f) {
  // an error left in the runtime's per-thread state by another caller's HIP
  // call must not be reported by this call's launch checks
  (void)hipGetLastError();
  try {
    return f();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return MGD_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return MGD_EHIP;
  } catch (...) {
    g_last_error = "unknown error";
    return MGD_EHIP;
  }
}
}  // namespace

// ===========================================================================
// Ctx
// ===========================================================================
namespace mgd {

const char* kernel_class_name(int c) {
  static const char* names[KC_COUNT] = {"spmv",        "block_matvec", "smooth_l0",
                                        "resid_l0",    "transfer_l0",  "vcycle_coarse",
                                        "coarse_solve", "orth",        "vec"};
  return (c >= 0 && c < KC_COUNT) ? names[c] : "?";
}

void* Ctx::dmalloc(size_t bytes) {
  void* p = nullptr;
  if (no_alloc)
    fail(MGD_EINVAL, "a device allocation of " + std::to_string(bytes) +
                         " bytes was requested inside a no-allocation call");
  if (has_alloc) {
    p = alloc.alloc(bytes, (void*)stream, alloc.user);
    if (!p) fail(MGD_ENOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
    return p;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(MGD_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}
void Ctx::dfree(void* p) {
  if (!p) return;
  if (has_alloc)
    alloc.free(p, (void*)stream, alloc.user);
  else
    (void)hipFree(p);
}
void* Ctx::host_stage(size_t bytes) {
  if (no_alloc && bytes > pinned_bytes) {
    // pageable static staging: no pinned allocation inside a no-allocation call
    alignas(256) static thread_local double stage[1024];
    MGD_REQUIRE(bytes <= sizeof(stage), "readback too large for a no-allocation call");
    return stage;
  }
  if (bytes > pinned_bytes) {
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    size_t sz = std::max<size_t>(bytes, 4096);
    MGD_HIP(hipHostMalloc(&pinned, sz, hipHostMallocDefault));
    pinned_bytes = sz;
  }
  return pinned;
}
hipEvent_t Ctx::take_event() {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  MGD_HIP(hipEventCreate(&e));
  return e;
}
void Ctx::prof_begin(int cls, hipEvent_t* a, hipStream_t s) {
  (void)cls;
  *a = take_event();
  MGD_HIP(hipEventRecord(*a, s));
}
void Ctx::prof_end(int cls, hipEvent_t a, double bytes_, double bytes_csr_, std::string kernel,
                   hipStream_t s) {
  hipEvent_t b = take_event();
  MGD_HIP(hipEventRecord(b, s));
  pending.push_back({cls, a, b, bytes_, bytes_csr_, std::move(kernel)});
  if (pending.size() > 4096) prof_collect();
}
void Ctx::prof_collect() {
  if (pending.empty()) return;
  MGD_HIP(hipStreamSynchronize(stream));
  for (auto& p : pending) {
    float ms_ = 0;
    MGD_HIP(hipEventElapsedTime(&ms_, p.a, p.b));
    launches[p.cls] += 1;
    ms[p.cls] += ms_;
    bytes[p.cls] += p.bytes;
    if (!p.kernel.empty()) {
      auto it = std::find_if(by_kernel.begin(), by_kernel.end(),
                             [&](const auto& kv) { return kv.first == p.kernel; });
      if (it == by_kernel.end()) {
        by_kernel.push_back({p.kernel, KernelStat{}});
        it = by_kernel.end() - 1;
      }
      it->second.launches += 1;
      it->second.ms += ms_;
      it->second.bytes += p.bytes;
      it->second.bytes_csr += p.bytes_csr;
    }
    event_pool.push_back(p.a);
    event_pool.push_back(p.b);
  }
  pending.clear();
}
Ctx::~Ctx() {
  gmres_ws.reset();  // its buffers go back through this context
  if (dev_err) dfree(dev_err);
  for (auto& p : pending) {
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  for (auto e : event_pool) hipEventDestroy(e);
  if (pinned) hipHostFree(pinned);
}

void check_csr_meta(const mgd_csr* A, bool square) {
  MGD_REQUIRE(A, "matrix is NULL");
  MGD_REQUIRE(A->n_rows >= 0 && A->n_cols >= 0 && A->nnz >= 0, "negative matrix size");
  MGD_REQUIRE(A->nnz < INT32_MAX, "nnz exceeds int32 indexing");
  MGD_REQUIRE(!square || A->n_rows == A->n_cols, "matrix must be square");
  MGD_REQUIRE(A->n_rows == 0 || A->row_ptr, "row_ptr is NULL");
  MGD_REQUIRE(A->nnz == 0 || (A->col_idx && A->val), "col_idx or val is NULL");
}

__global__ void k_validate(int n, int ncols, long long nnz, const int* __restrict__ rp,
                           const int* __restrict__ ci, int flags, int* __restrict__ bad) {
  const int require_diag = flags & 1, unsorted = flags & 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e0 = rp[i], e1 = rp[i + 1];
  if (i == 0 && e0 != 0) atomicOr(bad, 1);
  if (i == n - 1 && e1 != nnz) atomicOr(bad, 1);
  if (e1 < e0 || e0 < 0 || e1 > nnz) {
    atomicOr(bad, 1);
    return;
  }
  bool diag = false;
  for (int e = e0; e < e1; ++e) {
    const int j = ci[e];
    if (j < 0 || j >= ncols) atomicOr(bad, 2);
    if (!unsorted && e > e0 && ci[e - 1] >= j) atomicOr(bad, 4);
    if (j == i) diag = true;
  }
  if (require_diag && !diag) atomicOr(bad, 8);
}

static int csr_check_bits(Ctx* c, int n_rows, int n_cols, long long nnz, const int* rp,
                          const int* ci, bool require_diag, bool unsorted = false) {
  if (n_rows == 0) return 0;
  DBuf<int> bad(c, 1);
  fill<int>(c, bad.get(), 0, 1);
  hipLaunchKernelGGL(k_validate, dim3(cdiv(n_rows, 256)), dim3(256), 0, c->stream, n_rows, n_cols,
                     nnz, rp, ci, (require_diag ? 1 : 0) | (unsorted ? 2 : 0), bad.get());
  MGD_CHECK_LAUNCH();
  return read1(c, bad.get());
}

static std::string check_message(int b) {
  std::string m;
  if (b & 1) m += " row_ptr is not a monotone [0, nnz] sequence;";
  if (b & 2) m += " column index out of range;";
  if (b & 4) m += " columns not strictly ascending within a row;";
  if (b & 8) m += " a row does not store its diagonal entry;";
  return m;
}

void validate_csr_device(Ctx* c, const mgd_csr* A, bool require_diag) {
  const int b = csr_check_bits(c, A->n_rows, A->n_cols, (long long)A->nnz, A->row_ptr, A->col_idx,
                               require_diag);
  if (b) fail(MGD_EINVAL, "invalid CSR:" + check_message(b));
}

template <typename V>
void check_structure(Ctx* c, const Csr<V>& A, const char* what, bool require_diag) {
  const int b = csr_check_bits(c, A.n_rows, A.n_cols, A.nnz, A.rp.get(), A.ci.get(), require_diag);
  if (b)
    fail(MGD_EHIP, std::string("internal structure check failed for ") + what + ":" +
                       check_message(b) + step_suffix());
}
template void check_structure<double>(Ctx*, const Csr<double>&, const char*, bool);

void check_index_structure(Ctx* c, int n_rows, int n_cols, long long nnz, const int* rp,
                           const int* ci, const char* what) {
  const int b = csr_check_bits(c, n_rows, n_cols, nnz, rp, ci, false, true);
  if (b)
    fail(MGD_EHIP, std::string("internal structure check failed for ") + what + ":" +
                       check_message(b) + step_suffix());
}
template void check_structure<float>(Ctx*, const Csr<float>&, const char*, bool);

int* Ctx::err_flag() {
  if (!dev_err) {
    dev_err = static_cast<int*>(dmalloc(sizeof(int)));
    fill<int>(this, dev_err, 0, 1);
  }
  return dev_err;
}

void Ctx::check_device_errors(const char* where) {
  if (!dev_err) return;
  const int e = read1(this, dev_err);
  if (e) {
    fill<int>(this, dev_err, 0, 1);
    sync();
    fail(MGD_EHIP, std::string("device bounds check failed in ") + where + " (code " +
                       std::to_string(e) + ")" + step_suffix());
  }
}

void check_block_system(const mgd_block_system* A) {
  MGD_REQUIRE(A, "block system is NULL");
  MGD_REQUIRE(A->G >= 1 && A->G + 2 <= kMaxBlocks, "G must be in [1, 64]");
  MGD_REQUIRE(A->N >= 1, "N must be positive");
  MGD_REQUIRE((long long)(A->G + 2) * A->N < INT32_MAX, "system too large for int32 indices");
  MGD_REQUIRE(A->blocks, "blocks is NULL");
  MGD_REQUIRE(A->d_gE && A->d_Eg && A->d_EI && A->d_IE, "coupling pointer is NULL");
  for (int a = 0; a < A->G + 2; ++a) {
    check_csr_meta(&A->blocks[a], true);
    MGD_REQUIRE(A->blocks[a].n_rows == A->N, "every block must have N rows");
  }
}

BlockSysDev make_block_sys_dev(const mgd_block_system* A) {
  BlockSysDev S{};
  S.G = A->G;
  S.N = A->N;
  long long nnz = 0;
  for (int a = 0; a < A->G + 2; ++a) {
    S.blk[a] = {A->blocks[a].row_ptr, A->blocks[a].col_idx, A->blocks[a].val};
    S.nnz[a] = A->blocks[a].nnz;
    nnz += A->blocks[a].nnz;
  }
  S.tpr = default_tpr((double)nnz / ((double)(A->G + 2) * A->N));
  S.shared = 1;
  for (int a = 1; a < A->G + 2; ++a)
    if (A->blocks[a].row_ptr != A->blocks[0].row_ptr ||
        A->blocks[a].col_idx != A->blocks[0].col_idx || A->blocks[a].nnz != A->blocks[0].nnz)
      S.shared = 0;
  S.d_gE = A->d_gE;
  S.d_Eg = A->d_Eg;
  S.d_EI = A->d_EI;
  S.d_IE = A->d_IE;
  if (S.shared) attach_half_storage(A, S);
  return S;
}

}  // namespace mgd

// ===========================================================================
// exported functions
// ===========================================================================
extern "C" {

const char* mgd_last_error(void) { return g_last_error.c_str(); }
const char* mgd_version(void) { return "mgdamg 0.1 (gfx950)"; }

mgd_status mgd_ctx_create(int device, void* hip_stream, const mgd_allocator* allocator,
                          mgd_ctx** out) {
  return guard([&] {
    StepScope step_("mgd_ctx_create");
    MGD_REQUIRE(out, "out is NULL");
    int ndev = 0;
    MGD_HIP(hipGetDeviceCount(&ndev));
    MGD_REQUIRE(device >= 0 && device < ndev, "device ordinal out of range");
    auto c = std::make_unique<mgd_ctx>();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (allocator) {
      MGD_REQUIRE(allocator->alloc && allocator->free, "allocator callbacks are NULL");
      c->alloc = *allocator;
      c->has_alloc = true;
    }
    c->make_current();
    // MGD_XCD_ROWS=1: level kernels take contiguous row shares per chiplet
    const char* xr = std::getenv("MGD_XCD_ROWS");
    set_xcd_rows(xr && xr[0] == '1' ? 1 : 0);
    *out = c.release();
    return MGD_OK;
  });
}

mgd_status mgd_ctx_destroy(mgd_ctx* ctx) {
  return guard([&] {
    StepScope step_("mgd_ctx_destroy");
    if (!ctx) return MGD_OK;
    ctx->make_current();
    (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
    return MGD_OK;
  });
}

mgd_status mgd_ctx_synchronize(mgd_ctx* ctx) {
  return guard([&] {
    StepScope step_("mgd_ctx_synchronize");
    MGD_REQUIRE(ctx, "ctx is NULL");
    ctx->make_current();
    ctx->sync();
    return MGD_OK;
  });
}

mgd_status mgd_ctx_set_profiling(mgd_ctx* ctx, int enable) {
  return guard([&] {
    StepScope step_("mgd_ctx_set_profiling");
    MGD_REQUIRE(ctx, "ctx is NULL");
    ctx->make_current();
    if (!enable) ctx->prof_collect();
    ctx->profiling = enable != 0;
    return MGD_OK;
  });
}
mgd_status mgd_ctx_reset_kernel_stats(mgd_ctx* ctx) {
  return guard([&] {
    StepScope step_("mgd_ctx_reset_kernel_stats");
    MGD_REQUIRE(ctx, "ctx is NULL");
    ctx->make_current();
    ctx->prof_collect();
    for (int i = 0; i < KC_COUNT; ++i) {
      ctx->launches[i] = 0;
      ctx->ms[i] = 0;
      ctx->bytes[i] = 0;
    }
    ctx->by_kernel.clear();
    return MGD_OK;
  });
}
int mgd_kernel_class_count(void) { return KC_COUNT; }
const char* mgd_kernel_class_name(int cls) { return kernel_class_name(cls); }
mgd_status mgd_ctx_kernel_stats(mgd_ctx* ctx, int cls, int64_t* launches, double* total_ms,
                                double* total_bytes) {
  return guard([&] {
    StepScope step_("mgd_ctx_kernel_stats");
    MGD_REQUIRE(ctx, "ctx is NULL");
    MGD_REQUIRE(cls >= 0 && cls < KC_COUNT, "kernel class out of range");
    ctx->make_current();
    ctx->prof_collect();
    if (launches) *launches = ctx->launches[cls];
    if (total_ms) *total_ms = ctx->ms[cls];
    if (total_bytes) *total_bytes = ctx->bytes[cls];
    return MGD_OK;
  });
}

mgd_status mgd_ctx_kernel_symbol_count(mgd_ctx* ctx, int* count) {
  return guard([&] {
    StepScope step_("mgd_ctx_kernel_symbol_count");
    MGD_REQUIRE(ctx && count, "ctx or count is NULL");
    ctx->make_current();
    ctx->prof_collect();
    *count = (int)ctx->by_kernel.size();
    return MGD_OK;
  });
}
mgd_status mgd_ctx_kernel_symbol_stats(mgd_ctx* ctx, int index, char* name, int name_cap,
                                       int64_t* launches, double* total_ms, double* total_bytes,
                                       double* total_bytes_csr) {
  return guard([&] {
    StepScope step_("mgd_ctx_kernel_symbol_stats");
    MGD_REQUIRE(ctx, "ctx is NULL");
    MGD_REQUIRE(index >= 0 && index < (int)ctx->by_kernel.size(), "kernel index out of range");
    const auto& kv = ctx->by_kernel[index];
    if (name && name_cap > 0) {
      const size_t k = std::min<size_t>(kv.first.size(), (size_t)name_cap - 1);
      std::memcpy(name, kv.first.data(), k);
      name[k] = 0;
    }
    if (launches) *launches = kv.second.launches;
    if (total_ms) *total_ms = kv.second.ms;
    if (total_bytes) *total_bytes = kv.second.bytes;
    if (total_bytes_csr) *total_bytes_csr = kv.second.bytes_csr;
    return MGD_OK;
  });
}

mgd_status mgd_csr_spmv(mgd_ctx* ctx, const mgd_csr* A, const double* x, double* y) {
  return guard([&] {
    StepScope step_("mgd_csr_spmv");
    MGD_REQUIRE(ctx, "ctx is NULL");
    check_csr_meta(A, false);
    MGD_REQUIRE(A->n_rows == 0 || (x && y), "x or y is NULL");
    MGD_REQUIRE((const void*)x != (const void*)y, "x and y must not alias");
    ctx->make_current();
    CsrView<double> v{A->n_rows, A->n_cols, (int)A->nnz, A->row_ptr, A->col_idx, A->val};
    spmv(ctx, v, x, y, default_tpr(A->n_rows ? (double)A->nnz / A->n_rows : 1.0), KC_SPMV);
    return MGD_OK;
  });
}

void amg_params_default(amg_params* p) {
  if (!p) return;
  p->strength_theta = 0.25;
  p->dominance_theta = 0.9;
  p->seed = 1;
  p->max_levels = 25;
  p->coarse_max = 100;
  p->dense_max = 2000;
  p->n_pre = 1;
  p->n_post = 1;
  p->precision = 0;
  p->autotune = 0;
  p->coarsening = 0;
  p->hmis_tile = 1024;
  p->smoother = 0;
  p->aggressive_levels = 0;
}

static void check_amg_params(const amg_params* p) {
  MGD_REQUIRE(p, "params is NULL");
  MGD_REQUIRE(p->strength_theta > 0 && p->strength_theta < 1, "strength_theta must be in (0, 1)");
  MGD_REQUIRE(p->max_levels >= 1 && p->max_levels <= MGD_MAX_LEVELS, "max_levels out of range");
  MGD_REQUIRE(p->coarse_max >= 1, "coarse_max must be >= 1");
  MGD_REQUIRE(p->dense_max >= 1 && p->dense_max <= 8192, "dense_max must be in [1, 8192]");
  MGD_REQUIRE(p->n_pre >= 0 && p->n_post >= 0 && p->n_pre <= 16 && p->n_post <= 16,
              "n_pre / n_post out of range");
  MGD_REQUIRE(p->precision == 0 || p->precision == 1, "precision must be 0 or 1");
  MGD_REQUIRE(p->coarsening == 0 || p->coarsening == 1, "coarsening must be 0 (PMIS) or 1 (HMIS)");
  MGD_REQUIRE(p->coarsening == 0 || (p->hmis_tile >= 1 && p->hmis_tile <= 1024),
              "hmis_tile must be in [1, 1024]");
  MGD_REQUIRE(p->smoother == 0 || p->smoother == 1, "smoother must be 0 (CF-l1-Jacobi) or 1 (MC-GS)");
  MGD_REQUIRE(p->aggressive_levels >= 0 && p->aggressive_levels <= MGD_MAX_LEVELS,
              "aggressive_levels must be in [0, MGD_MAX_LEVELS]");
}

mgd_status amg_setup(mgd_ctx* ctx, const mgd_csr* A, const amg_params* p, amg_hierarchy** out) {
  return guard([&] {
    StepScope step_("amg_setup");
    MGD_REQUIRE(ctx && out, "ctx or out is NULL");
    check_amg_params(p);
    check_csr_meta(A, true);
    MGD_REQUIRE(A->n_rows >= 1, "matrix is empty");
    ctx->make_current();
    validate_csr_device(ctx, A, true);
    StepScope st_copy("amg_setup: input copy");
    auto t0 = std::chrono::steady_clock::now();
    auto h = std::make_unique<amg_hierarchy>();
    h->ctx = ctx;
    h->prm = *p;
    h->n = A->n_rows;
    Csr<double> M;
    csr_copy_from(ctx, A, M);
    check_structure(ctx, M, "copied input matrix", true);
    amg_build(ctx, std::move(M), h->prm, h->H);
    if (p->precision == 0)
      h->union64();
    else
      h->union32();
    ctx->sync();
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h.release();
    return MGD_OK;
  });
}

mgd_status amg_apply(mgd_ctx* ctx, amg_hierarchy* h, const double* r, double* z, int n_cycles) {
  return guard([&] {
    StepScope step_("amg_apply");
    MGD_REQUIRE(ctx && h, "ctx or hierarchy is NULL");
    MGD_REQUIRE(h->ctx == ctx, "hierarchy belongs to another context");
    MGD_REQUIRE(r && z && (const void*)r != (const void*)z, "r, z must be distinct and non-NULL");
    MGD_REQUIRE(n_cycles >= 1, "n_cycles must be >= 1");
    ctx->make_current();
    h->apply(r, z, n_cycles);
    return MGD_OK;
  });
}

mgd_status amg_get_info(const amg_hierarchy* h, amg_info* out) {
  return guard([&] {
    StepScope step_("amg_get_info");
    MGD_REQUIRE(h && out, "hierarchy or out is NULL");
    *out = amg_info{};
    out->levels = (int)h->H.levels.size();
    out->coarse_kind = h->H.coarse_kind;
    double gs = 0, os_ = 0;
    for (size_t l = 0; l < h->H.levels.size(); ++l) {
      const auto& L = h->H.levels[l];
      out->n[l] = L.A.n_rows;
      out->nnz[l] = L.A.nnz;
      out->nnz_P[l] = L.P.nnz;
      out->pmis_rounds[l] = L.pmis_rounds;
      gs += L.A.n_rows;
      os_ += L.A.nnz;
    }
    out->grid_complexity = gs / std::max(1, h->H.levels[0].A.n_rows);
    out->operator_complexity = os_ / std::max(1, h->H.levels[0].A.nnz);
    return MGD_OK;
  });
}

mgd_status amg_export_level(mgd_ctx* ctx, const amg_hierarchy* h, int level, int8_t* cf,
                            int32_t* a_row_ptr, int32_t* a_col, double* a_val, int32_t* p_row_ptr,
                            int32_t* p_col, double* p_val) {
  return guard([&] {
    StepScope step_("amg_export_level");
    MGD_REQUIRE(ctx && h, "ctx or hierarchy is NULL");
    MGD_REQUIRE(level >= 0 && level < (int)h->H.levels.size(), "level out of range");
    ctx->make_current();
    const auto& L = h->H.levels[level];
    const int n = L.A.n_rows;
    if (cf) {
      if (L.cf.p)
        copy_d2h(ctx, cf, L.cf.get(), (size_t)n);
      else
        std::fill(cf, cf + n, (int8_t)0);
    }
    if (a_row_ptr) copy_d2h(ctx, a_row_ptr, L.A.rp.get(), (size_t)n + 1);
    if (a_col) copy_d2h(ctx, a_col, L.A.ci.get(), (size_t)L.A.nnz);
    if (a_val) copy_d2h(ctx, a_val, L.A.v.get(), (size_t)L.A.nnz);
    if (L.P.rp.p) {
      if (p_row_ptr) copy_d2h(ctx, p_row_ptr, L.P.rp.get(), (size_t)n + 1);
      if (p_col) copy_d2h(ctx, p_col, L.P.ci.get(), (size_t)L.P.nnz);
      if (p_val) copy_d2h(ctx, p_val, L.P.v.get(), (size_t)L.P.nnz);
    }
    return MGD_OK;
  });
}

mgd_status amg_destroy(amg_hierarchy* h) {
  return guard([&] {
    StepScope step_("amg_destroy");
    if (h) {
      h->ctx->make_current();
      h->ctx->sync();
      delete h;
    }
    return MGD_OK;
  });
}

mgd_status mgd_block_matvec(mgd_ctx* ctx, const mgd_block_system* A, const double* x, double* y) {
  return guard([&] {
    StepScope step_("mgd_block_matvec");
    MGD_REQUIRE(ctx, "ctx is NULL");
    check_block_system(A);
    MGD_REQUIRE(x && y && (const void*)x != (const void*)y, "x, y must be distinct and non-NULL");
    ctx->make_current();
    block_matvec(ctx, make_block_sys_dev(A), x, nullptr, y);
    return MGD_OK;
  });
}

mgd_status mgd_assemble(mgd_ctx* ctx, const mgd_coeffs* c, mgd_block_system* out) {
  return guard([&] {
    StepScope step_("mgd_assemble");
    MGD_REQUIRE(ctx && out, "ctx or out is NULL");
    ctx->make_current();
    assemble_impl(ctx, c, out);
    return MGD_OK;
  });
}

mgd_status mgd_block_system_transpose(mgd_ctx* ctx, const mgd_block_system* A,
                                      mgd_block_system* out) {
  return guard([&] {
    StepScope step_("mgd_block_system_transpose");
    MGD_REQUIRE(ctx && out, "ctx or out is NULL");
    check_block_system(A);
    ctx->make_current();
    system_transpose_impl(ctx, A, out);
    return MGD_OK;
  });
}

mgd_status mgd_block_system_free(mgd_ctx* ctx, mgd_block_system* s) {
  return guard([&] {
    StepScope step_("mgd_block_system_free");
    MGD_REQUIRE(ctx && s, "ctx or system is NULL");
    ctx->make_current();
    ctx->sync();
    system_free_impl(s);
    return MGD_OK;
  });
}

void block_params_default(block_params* p) {
  if (!p) return;
  p->kind = MGD_PC_SCHUR2;
  amg_params_default(&p->amg);
  p->cycles_rad = p->cycles_E = p->cycles_I = 1;
  p->pctl_p_tol = 1e-2;
  p->pctl_p_maxcycles = 100;
  p->batched = 0;
  p->use_graph = 0;
  p->transpose = 0;
  p->adaptive = 0;
  p->theta_wc = 1e-2;
  p->sigma_wc = 0.5;
  p->theta_wd = 0.9;
  p->jacobi_sweeps = 2;
  p->inner_tol = 0.0;
  p->inner_maxcycles = 100;
  p->option4_steps = 0;
}

mgd_status block_precond_create(mgd_ctx* ctx, const mgd_block_system* A, const block_params* p,
                                block_precond** out) {
  return guard([&] {
    StepScope step_("block_precond_create");
    MGD_REQUIRE(ctx && p && out, "ctx, params or out is NULL");
    check_block_system(A);
    check_amg_params(&p->amg);
    MGD_REQUIRE(p->pctl_p_tol > 0 && p->pctl_p_maxcycles >= 1, "bad PCTL inner tolerance");
    MGD_REQUIRE(p->adaptive == 0 || p->adaptive == 1, "adaptive must be 0 or 1");
    MGD_REQUIRE(p->inner_tol >= 0 && p->inner_tol < 1, "inner_tol must be in [0, 1)");
    MGD_REQUIRE(p->inner_maxcycles >= 1 && p->inner_maxcycles <= 1000,
                "inner_maxcycles must be in [1, 1000]");
    MGD_REQUIRE(p->option4_steps >= 0 && p->option4_steps <= 100,
                "option4_steps must be in [0, 100]");
    MGD_REQUIRE(p->option4_steps == 0 || p->kind == MGD_PC_SCHUR1 || p->kind == MGD_PC_SCHUR2,
                "option #4 applies to SCHUR1 (C_E) and SCHUR2 (S_I)");
    if (p->adaptive) {
      MGD_REQUIRE(p->kind == MGD_PC_PCTL || p->kind == MGD_PC_SCHUR1 || p->kind == MGD_PC_SCHUR2,
                  "the adaptive strategy applies to PCTL, SCHUR1 and SCHUR2");
      MGD_REQUIRE(p->theta_wc > 0 && p->theta_wc < 1 && p->sigma_wc >= 0 && p->sigma_wc <= 1 &&
                      p->theta_wd > 0 && p->theta_wd < 1,
                  "adaptive thresholds out of range (theta_wc, theta_wd in (0,1), sigma_wc in [0,1])");
      MGD_REQUIRE(p->jacobi_sweeps >= 1 && p->jacobi_sweeps <= 64, "jacobi_sweeps must be in [1, 64]");
    }
    ctx->make_current();
    for (int a = 0; a < A->G + 2; ++a) validate_csr_device(ctx, &A->blocks[a], true);
    *out = block_precond_create_impl(ctx, A, p);
    return MGD_OK;
  });
}

mgd_status block_precond_apply(mgd_ctx* ctx, block_precond* M, const double* r, double* z) {
  return guard([&] {
    StepScope step_("block_precond_apply");
    MGD_REQUIRE(ctx && M, "ctx or preconditioner is NULL");
    MGD_REQUIRE(M->ctx == ctx, "preconditioner belongs to another context");
    MGD_REQUIRE(r && z && (const void*)r != (const void*)z, "r, z must be distinct and non-NULL");
    ctx->make_current();
    block_precond_apply_dispatch(M, r, z);
    return MGD_OK;
  });
}

mgd_status block_precond_get_info(const block_precond* M, block_precond_info* out) {
  return guard([&] {
    StepScope step_("block_precond_get_info");
    MGD_REQUIRE(M && out, "preconditioner or out is NULL");
    *out = block_precond_info{};
    out->kind = M->prm.kind;
    int nh = 0;
    for (auto& h : M->hier) nh += h ? 1 : 0;
    out->n_hierarchies = nh;
    out->inverses_per_apply = M->inverses_last;
    out->matvecs_per_apply = M->matvecs_last;
    for (size_t i = 0; i < M->p_cycles.size() && i < 66; ++i) out->pctl_p_cycles[i] = M->p_cycles[i];
    out->setup_ms = M->setup_ms;
    for (int r = 0; r < 66; ++r) out->wd_count[r] = -1;
    for (int r = 0; r < 66; ++r)
      out->inner_cycles[r] = r < (int)M->inner_cycles.size() ? M->inner_cycles[r] : -1;
    if (M->prm.adaptive) {
      for (int g = 0; g < M->G && g < 64; ++g) {
        out->wc_count_gE[g] = M->cnt_gE[g];
        out->wc_count_Eg[g] = M->cnt_Eg[g];
        out->weak_gE[g] = M->weak_gE[g];
        out->weak_Eg[g] = M->weak_Eg[g];
      }
      out->wc_count_EI = M->cnt_EI;
      out->wc_count_IE = M->cnt_IE;
      out->weak_EI = M->weak_EI;
      out->weak_IE = M->weak_IE;
      for (size_t r = 0; r < M->wd_count.size() && r < 66; ++r) {
        out->wd_count[r] = M->wd_count[r];
        out->jacobi[r] = M->jacobi[r];
      }
    }
    return MGD_OK;
  });
}

mgd_status block_precond_get_hierarchy(const block_precond* M, int index, const amg_hierarchy** out) {
  return guard([&] {
    StepScope step_("block_precond_get_hierarchy");
    MGD_REQUIRE(M && out, "preconditioner or out is NULL");
    MGD_REQUIRE(index >= 0 && index < (int)M->hier.size() && M->hier[index],
                "no hierarchy at this index");
    *out = M->hier[index].get();
    return MGD_OK;
  });
}

mgd_status block_precond_destroy(block_precond* M) {
  return guard([&] {
    StepScope step_("block_precond_destroy");
    if (M) {
      M->ctx->make_current();
      M->ctx->sync();
      delete M;
    }
    return MGD_OK;
  });
}

void gmres_params_default(gmres_params* p) {
  if (!p) return;
  p->restart = 30;
  p->max_iters = 1000;
  p->rtol = 1e-8;
  p->flexible = 1;
  p->profile = 0;
}

mgd_status gmres_solve(mgd_ctx* ctx, const mgd_block_system* A, block_precond* M, const double* b,
                       double* x, const gmres_params* p, gmres_result* out) {
  return guard([&] {
    StepScope step_("gmres_solve");
    MGD_REQUIRE(ctx && p && out, "ctx, params or result is NULL");
    check_block_system(A);
    MGD_REQUIRE(b && x && (const void*)b != (const void*)x, "b, x must be distinct and non-NULL");
    MGD_REQUIRE(!M || M->ctx == ctx, "preconditioner belongs to another context");
    MGD_REQUIRE(!M || (M->G == A->G && M->N == A->N), "preconditioner built for another shape");
    MGD_REQUIRE(p->rtol >= 0, "rtol must be >= 0");
    ctx->make_current();
    const mgd_status st = gmres_impl(ctx, make_block_sys_dev(A), M, b, x, *p, *out);
    ctx->check_device_errors("gmres_solve (V-cycle tail barrier)");
    return st;
  });
}

mgd_status gmres_solve_noalloc(mgd_ctx* ctx, const mgd_block_system* A, block_precond* M,
                               const double* b, double* x, const gmres_params* p,
                               gmres_result* out) {
  return guard([&] {
    StepScope step_("gmres_solve_noalloc");
    MGD_REQUIRE(ctx && p && out, "ctx, params or result is NULL");
    check_block_system(A);
    MGD_REQUIRE(b && x && (const void*)b != (const void*)x, "b, x must be distinct and non-NULL");
    MGD_REQUIRE(!M || M->ctx == ctx, "preconditioner belongs to another context");
    MGD_REQUIRE(!M || (M->G == A->G && M->N == A->N), "preconditioner built for another shape");
    MGD_REQUIRE(p->rtol >= 0, "rtol must be >= 0");
    MGD_REQUIRE(!p->profile, "per-phase profiling is not available in a no-allocation call");
    ctx->make_current();
    struct NoAlloc {  // restores the context's mode on every exit
      Ctx* c;
      explicit NoAlloc(Ctx* c_) : c(c_) { c->no_alloc = true; }
      ~NoAlloc() { c->no_alloc = false; }
    } na(ctx);
    const mgd_status st = gmres_impl(ctx, make_block_sys_dev(A), M, b, x, *p, *out);
    ctx->check_device_errors("gmres_solve_noalloc (V-cycle tail barrier)");
    return st;
  });
}

mgd_status mgd_adjoint_gradients(mgd_ctx* ctx, const mgd_coeffs* c, const double* x,
                                 const double* lambda, double* dL_dkappa, double* dL_dc) {
  return guard([&] {
    StepScope step_("mgd_adjoint_gradients");
    MGD_REQUIRE(ctx && x && lambda, "ctx, x or lambda is NULL");
    ctx->make_current();
    adjoint_gradients_impl(ctx, c, x, lambda, dL_dkappa, dL_dc);
    ctx->sync();
    return MGD_OK;
  });
}

mgd_status adjoint_solve(mgd_ctx* ctx, const mgd_coeffs* c, const mgd_block_system* A,
                         block_precond* M_T, const double* x, const double* g, double* lambda,
                         double* dL_dkappa, double* dL_dc, const gmres_params* p,
                         gmres_result* out) {
  return guard([&] {
    StepScope step_("adjoint_solve");
    MGD_REQUIRE(ctx && p && out && x && g && lambda, "NULL argument");
    check_block_system(A);
    check_coeffs(c);
    MGD_REQUIRE(!M_T || M_T->prm.transpose, "M_T must be created with transpose = 1");
    ctx->make_current();
    mgd_block_system AT{};
    system_transpose_impl(ctx, A, &AT);
    mgd_status st;
    try {
      fill<double>(ctx, lambda, 0.0, (size_t)(A->G + 2) * A->N);
      st = gmres_impl(ctx, make_block_sys_dev(&AT), M_T, g, lambda, *p, *out);
    } catch (...) {
      system_free_impl(&AT);
      throw;
    }
    system_free_impl(&AT);
    if (st != MGD_OK && st != MGD_ENOTCONV) return st;
    adjoint_gradients_impl(ctx, c, x, lambda, dL_dkappa, dL_dc);
    ctx->sync();
    ctx->check_device_errors("adjoint_solve (V-cycle tail barrier)");
    if (st == MGD_ENOTCONV) g_last_error = "adjoint GMRES reached max_iters";
    return st;
  });
}

}  // extern "C"
