// Internal runtime shared by every translation unit of libmgdamg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <initializer_list>
#include <memory>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mgdamg.h"

namespace mgd {

// ---------------------------------------------------------------------------
// errors: internal code throws Error; the C ABI converts it to a status.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  mgd_status code;
  Error(mgd_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(mgd_status c, const std::string& m) { throw Error(c, m); }

// The library step in progress on this thread (set by StepScope); HIP errors
// name it, so an asynchronous device fault reported at a later synchronisation
// still says which step's kernels were in flight.
inline std::string& current_step() {
  static thread_local std::string s;
  return s;
}
struct StepScope {
  std::string prev;
  explicit StepScope(const std::string& step) : prev(current_step()) { current_step() = step; }
  ~StepScope() { current_step() = prev; }
};
inline std::string step_suffix() {
  return current_step().empty() ? std::string() : " [step: " + current_step() + "]";
}

#define MGD_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      ::mgd::fail(e_ == hipErrorOutOfMemory ? MGD_ENOMEM : MGD_EHIP,                      \
                  std::string(#call) + ": " + hipGetErrorString(e_) + " (" __FILE__ ")" + \
                      ::mgd::step_suffix());                                              \
  } while (0)

#define MGD_CHECK_LAUNCH() MGD_HIP(hipGetLastError())

#define MGD_REQUIRE(cond, msg)                              \
  do {                                                      \
    if (!(cond)) ::mgd::fail(MGD_EINVAL, std::string(msg)); \
  } while (0)

// ---------------------------------------------------------------------------
// kernel classes for the optional per-class event timing
// ---------------------------------------------------------------------------
enum KernelClass : int {
  KC_SPMV = 0,       // plain y = A x (block diagonal or monolithic)
  KC_BLOCK_MATVEC,   // eq. 2.2 block matvec / residual
  KC_SMOOTH_L0,      // CF-l1-Jacobi half-sweep, finest level
  KC_RESID_L0,       // residual, finest level
  KC_TRANSFER_L0,    // restriction + prolongation, finest level
  KC_VCYCLE_COARSE,  // every V-cycle kernel below the finest level
  KC_COARSE_SOLVE,   // dense coarsest solve
  KC_ORTH,           // GMRES orthogonalisation / norms / updates
  KC_VEC,            // vector glue (Hadamard products, casts, copies)
  KC_COUNT
};
const char* kernel_class_name(int c);

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  mgd_allocator alloc{};
  bool has_alloc = false;
  // pinned host staging for small readbacks
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  // GMRES basis and scratch kept between calls of the same size (allocation
  // stays out of the solve, and graph-replayed steps find the same buffers)
  std::shared_ptr<void> gmres_ws;
  // profiling
  bool profiling = false;
  // set for the duration of a no-allocation call: any device allocation is an
  // error, small readbacks stage through static host memory, and the solve
  // runs as direct launches (no graph instantiation, no second stream)
  bool no_alloc = false;
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes;        // algorithmic bytes in the stored layout
    double bytes_csr;    // the same launch priced as plain CSR with 32-bit indices
    std::string kernel;  // symbol of the single kernel timed, or empty
  };
  struct KernelStat {
    int64_t launches = 0;
    double ms = 0, bytes = 0, bytes_csr = 0;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  int* dev_err = nullptr;  // set by in-kernel bounds checks
  int64_t launches[KC_COUNT] = {};
  double ms[KC_COUNT] = {};
  double bytes[KC_COUNT] = {};
  std::vector<std::pair<std::string, KernelStat>> by_kernel;  // first-seen order

  void* dmalloc(size_t bytes);
  void dfree(void* p);
  void* host_stage(size_t bytes);  // pinned buffer of at least `bytes`
  void sync() { MGD_HIP(hipStreamSynchronize(stream)); }
  void make_current() { MGD_HIP(hipSetDevice(device)); }
  int* err_flag();                           // device int, zero until a check fails
  void check_device_errors(const char* where);  // synchronises; throws when set
  // profiling hooks
  hipEvent_t take_event();
  void prof_begin(int cls, hipEvent_t* a, hipStream_t s);
  void prof_end(int cls, hipEvent_t a, double bytes, double bytes_csr, std::string kernel,
                hipStream_t s);
  void prof_collect();  // synchronises
  ~Ctx();
};

// RAII scope: events around one launch (or a short fixed sequence) when
// profiling is on.  `kernel` names the kernel symbol when the scope holds
// exactly one launch, so per-kernel averages can be compared with a trace.
// bytes: algorithmic bytes of the launch in its stored layout; bytes_csr: the
// same launch priced as plain CSR (value and 4-byte column per entry, 4-byte
// row pointer per row swept), which equals bytes where no matrix is read.
// The events go on `stream` (default: the context stream), the stream the
// timed launch runs on.
struct ProfScope {
  Ctx* c;
  int cls;
  double bytes, bytes_csr;
  std::string kernel;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(Ctx* c_, int cls_, double bytes_, std::string kernel_ = std::string(),
            double bytes_csr_ = -1.0, hipStream_t stream = nullptr)
      : c(c_), cls(cls_), bytes(bytes_), bytes_csr(bytes_csr_ < 0 ? bytes_ : bytes_csr_),
        kernel(std::move(kernel_)), s(stream ? stream : c_->stream) {
    if (c->profiling) c->prof_begin(cls, &a, s);
  }
  ~ProfScope() {
    if (c->profiling && a) c->prof_end(cls, a, bytes, bytes_csr, std::move(kernel), s);
  }
};

// Kernel symbol with template arguments as a demangler prints them
// ("k_half<float, 1>"); empty unless profiling, so launches pay nothing.
template <typename T>
inline const char* type_name() {
  return sizeof(T) == 4 ? "float" : "double";
}
inline std::string ksym(const Ctx* c, const char* base, std::initializer_list<std::string> args) {
  if (!c->profiling) return std::string();
  std::string s(base);
  const char* sep = "<";
  for (const auto& a : args) {
    s += sep;
    s += a;
    sep = ", ";
  }
  return args.size() ? s + ">" : s;
}


// ---------------------------------------------------------------------------
// device buffer owned through the context allocator
// ---------------------------------------------------------------------------
template <typename T>
struct DBuf {
  Ctx* ctx = nullptr;
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(Ctx* c, size_t count) { alloc(c, count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { swap(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    reset();
    swap(o);
    return *this;
  }
  ~DBuf() { reset(); }
  void swap(DBuf& o) noexcept {
    std::swap(ctx, o.ctx);
    std::swap(p, o.p);
    std::swap(n, o.n);
  }
  void alloc(Ctx* c, size_t count) {
    reset();
    ctx = c;
    n = count;
    p = count ? static_cast<T*>(c->dmalloc(count * sizeof(T))) : nullptr;
  }
  void reset() {
    if (p && ctx) ctx->dfree(p);
    p = nullptr;
    n = 0;
  }
  T* get() const { return p; }
  size_t bytes() const { return n * sizeof(T); }
};

template <typename T>
inline void copy_d2h(Ctx* c, T* h, const T* d, size_t n) {
  if (!n) return;
  MGD_HIP(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, c->stream));
  c->sync();
}
template <typename T>
inline void copy_h2d(Ctx* c, T* d, const T* h, size_t n) {
  if (!n) return;
  MGD_HIP(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, c->stream));
  c->sync();
}
// Device-to-device copies run as a library kernel on the context stream.
void device_copy(Ctx* c, void* dst, const void* src, size_t bytes);
template <typename T>
inline void copy_d2d(Ctx* c, T* d, const T* s, size_t n) {
  if (!n) return;
  device_copy(c, d, s, n * sizeof(T));
}
// Read a single device value (synchronises).
template <typename T>
inline T read1(Ctx* c, const T* d) {
  T* h = static_cast<T*>(c->host_stage(sizeof(T)));
  MGD_HIP(hipMemcpyAsync(h, d, sizeof(T), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  return *h;
}

// ---------------------------------------------------------------------------
// device CSR (owned)
// ---------------------------------------------------------------------------
template <typename V>
struct Csr {
  int n_rows = 0, n_cols = 0, nnz = 0;
  DBuf<int> rp, ci;
  DBuf<V> v;
  void alloc(Ctx* c, int nr, int nc, int nz) {
    n_rows = nr;
    n_cols = nc;
    nnz = nz;
    rp.alloc(c, (size_t)nr + 1);
    ci.alloc(c, (size_t)nz);
    v.alloc(c, (size_t)nz);
  }
};

// Non-owning view used by kernels/launchers.
template <typename V>
struct CsrView {
  int n_rows, n_cols, nnz;
  const int* rp;
  const int* ci;
  const V* v;
};
template <typename V>
inline CsrView<V> view(const Csr<V>& a) {
  return {a.n_rows, a.n_cols, a.nnz, a.rp.get(), a.ci.get(), a.v.get()};
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// Structural check of an internal CSR on the device (row_ptr monotone in
// [0, nnz], columns in range and strictly ascending, diagonal when asked);
// throws MGD_EHIP naming `what` when a library-built structure is malformed.
template <typename V>
void check_structure(Ctx* c, const Csr<V>& A, const char* what, bool require_diag);

// Same for an index structure whose rows need not be sorted.
void check_index_structure(Ctx* c, int n_rows, int n_cols, long long nnz, const int* rp,
                           const int* ci, const char* what);

// Validate a caller CSR (host-side metadata only; device contents are
// trusted to be sorted as documented, and checked by validate_csr_device).
void check_csr_meta(const mgd_csr* A, bool square);
// Device-side structural validation (sorted columns in range, row_ptr monotone,
// diagonal present when require_diag).  Synchronises.
void validate_csr_device(Ctx* c, const mgd_csr* A, bool require_diag);

}  // namespace mgd

struct mgd_ctx : mgd::Ctx {};
