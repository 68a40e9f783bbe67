// Launchers shared between translation units.  All enqueue on ctx->stream.
#pragma once
#include <functional>

#include "common.hpp"

namespace mgd {

constexpr int kBlock = 256;     // default workgroup size (4 wavefronts of 64)
constexpr int kRedBlocks = 1024; // fixed partial count of deterministic reductions

// ---- scans (int32) -----------------------------------------------------------
// out[0..n]: out[i] = sum_{j<i} in[j], out[n] = total.  No synchronisation.
void exclusive_scan(Ctx* c, const int* in, int* out, int n);
// Same, then returns the total (synchronises).
int exclusive_scan_total(Ctx* c, const int* in, int* out, int n);

// ---- fills / casts ---------------------------------------------------------
template <typename T>
void fill(Ctx* c, T* p, T v, size_t n);
template <typename D, typename S>
void cast_copy(Ctx* c, D* dst, const S* src, size_t n, int cls);

// ---- deterministic reductions (fixed partition, fixed order) ---------------
struct RedWork {
  DBuf<double> partial;  // kRedBlocks * 66
  void ensure(Ctx* c) {
    if (!partial.p) partial.alloc(c, (size_t)kRedBlocks * 66);
  }
};
// out[0] = sum x_i y_i  (device scalar)
void dot_dev(Ctx* c, RedWork& w, const double* x, const double* y, size_t n, double* out);
// Arnoldi orthogonalisation of w against V_0..V_{J-1} (rows of stride ldv),
// classical Gram-Schmidt with selective reorthogonalisation (J < 32):
//   mdot_dev:        h[i] = V_i . w (i < J), h[J] = w . w
//   update_mdot_dev: w -= sum h_i V_i; h2[i] = V_i . w_new, h2[J] = w_new . w_new
//   orth_finish_dev: hcol[0..J-1] = h1 (+ h2 when h2[J] < h1[J] / 2, the second
//                    projection then applied: w -= sum h2_i V_i), hcol[J] = the
//                    scale (the norm, by Pythagoras after the second projection),
//                    hcol[J+1] = 1 if it ran; w /= hcol[J] in place, and
//                    hcol[J+2] = the exact squared norm of w before the scaling
void mdot_dev(Ctx* c, RedWork& w, const double* V, size_t ldv, int J, const double* wv, size_t n,
              double* h);
void update_mdot_dev(Ctx* c, RedWork& w, const double* V, size_t ldv, int J, const double* h,
                     double* wv, size_t n, double* h2);
void orth_finish_dev(Ctx* c, RedWork& w, const double* V, size_t ldv, int J, const double* h1,
                     const double* h2, double* hcol, double* wv, size_t n);
// One Arnoldi step of classical Gram-Schmidt with delayed reorthogonalisation
// (two sweeps over the basis).  V_0..V_{F-1} are final; vj (or null) is the
// previous step's vector, orthogonalised once and scaled, still to be
// reorthogonalised; w = A z_j.  Writes coef (device, kDcgsCoef doubles):
//   [0, 32) a = V_k . vj, [32, 64) h = the projection of w on the final basis
//   (V_0..V_{F-1}, then the corrected vj when present), [64] beta, the norm
//   of vj - sum a_k V_k by Pythagoras, [65] alpha, the norm of w - sum h_k v_k
//   by Pythagoras (1 when not positive), [66] and [67] the exact squared norms
//   of the corrected vj (after division by beta) and of w before its division
//   by alpha.  vj <- (vj - sum a_k V_k) / beta in place; w <- (w - ...) / alpha.
constexpr int kDcgsCoef = 68;
// With `split`, the update sweep runs first over entries [lo, hi), then over
// the rest on the `side` stream while `beside` enqueues other work on
// ctx->stream; both are joined before [66] and [67] are summed.  The vectors
// are the same as without it; [66] and [67] are summed in another order.
struct DcgsSplit {
  size_t lo = 0, hi = 0;
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::function<void()> beside;
};
void dcgs_step_dev(Ctx* c, RedWork& w, const double* V, size_t ldv, int F, double* vj,
                   double* wv, size_t n, double* dots, double* coef,
                   const DcgsSplit* split = nullptr);
// v *= a
void scale_dev(Ctx* c, double a, double* v, size_t n);
// x += sum_i y_i Z_i (y on device)
void combine_dev(Ctx* c, const double* Z, size_t ldz, int K, const double* y, double* x, size_t n);
// y = b - y (in place, residual from a matvec result)
void rsub(Ctx* c, const double* b, double* y, size_t n);
// y = a * x
void scale_copy(Ctx* c, double* y, const double* x, double a, size_t n);
void axpy(Ctx* c, double* y, const double* x, double a, size_t n);

// ---- sparse ------------------------------------------------------------------
// y = A x (FP64), row groups of `tpr` lanes (1..64, power of two).
void spmv(Ctx* c, const CsrView<double>& A, const double* x, double* y, int tpr, int cls);

}  // namespace mgd
