// Block preconditioners of Section 3: monolithic AMG, block-diagonal, PCTL
// (Section 3.2, coarse operator eq. 3.1), Schur1 and Schur2 (Section 3.3)
// with the diagonal Schur-complement approximations of Section 3.4, and the
// elimination-only factor of Schur2.  The independent scalar V-cycles of a
// step run either as one batched set of launches over a union of
// hierarchies or one hierarchy after another.
#pragma clang fp contract(off)

#include <chrono>
#include <cstdlib>
#include <functional>

#include "handles.hpp"
#include "kernels.hpp"
#include "rowdot.hpp"

using namespace mgd;

// ===========================================================================
// amg_hierarchy helpers
// ===========================================================================
Union<double>* amg_hierarchy::union64() {
  if (!u64) {
    std::vector<const SetupHierarchy*> m{&H};
    u64 = build_union<double>(ctx, m, prm.n_pre, prm.n_post, prm.autotune, prm.smoother);
  }
  return u64.get();
}
Union<float>* amg_hierarchy::union32() {
  if (!u32) {
    std::vector<const SetupHierarchy*> m{&H};
    u32 = build_union<float>(ctx, m, prm.n_pre, prm.n_post, prm.autotune, prm.smoother);
  }
  return u32.get();
}
void amg_hierarchy::apply(const double* r, double* z, int cycles) {
  if (prm.precision == 0) {
    union64()->apply(ctx, r, z, cycles);
    return;
  }
  Union<float>* u = union32();
  if (in32.n < (size_t)n) {
    in32.alloc(ctx, (size_t)n);
    out32.alloc(ctx, (size_t)n);
  }
  cast_copy<float, double>(ctx, in32.get(), r, (size_t)n, KC_VEC);
  u->apply(ctx, in32.get(), out32.get(), cycles);
  cast_copy<double, float>(ctx, z, out32.get(), (size_t)n, KC_VEC);
}

template <typename T>
static Union<T>* union_of(amg_hierarchy* h);
template <>
Union<double>* union_of<double>(amg_hierarchy* h) {
  return h->union64();
}
template <>
Union<float>* union_of<float>(amg_hierarchy* h) {
  return h->union32();
}

// ===========================================================================
// glue kernels
// ===========================================================================
namespace mgd {

template <typename T>
__global__ void k_group_in(int N, const SegIn* __restrict__ tab, const double* __restrict__ r,
                           const T* __restrict__ w, T* __restrict__ in) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const SegIn d = tab[blockIdx.y];
  double v = r[(size_t)d.seg * N + i];
  if (d.coef) v = v - d.coef[i] * (double)w[i];
  in[(size_t)blockIdx.y * N + i] = (T)v;
}

template <typename T, bool SUM>
__global__ void k_group_out(int N, int nm, const SegOut* __restrict__ tab, const T* __restrict__ out,
                            double* __restrict__ z, T* __restrict__ sT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  // four members at a time: their loads in flight together, the sum in member order
  for (int m0 = 0; m0 < nm; m0 += 4) {
    double x[4], cf[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (m0 + q < nm) {
        const SegOut d = tab[m0 + q];
        x[q] = (double)out[(size_t)(m0 + q) * N + i];
        cf[q] = (SUM && d.coef) ? d.coef[i] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (m0 + q < nm) {
        const SegOut d = tab[m0 + q];
        z[(size_t)d.seg * N + i] = x[q];
        if (SUM && d.coef) s = s + cf[q] * x[q];
      }
    }
  }
  if (SUM) sT[i] = (T)s;
}

// the same from a union's result left in stored order: member m's row i read
// at its stored position (C, F or dense region), the arithmetic unchanged
template <typename T, bool SUM>
__global__ void k_group_out_st(int N, int nm, const SegOut* __restrict__ tab, StoredOut<T> so,
                               double* __restrict__ z, T* __restrict__ sT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = 0.0;
  for (int m0 = 0; m0 < nm; m0 += 4) {
    int k[4];
    double x[4], cf[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (m0 + q < nm) {
        const SegOut d = tab[m0 + q];
        k[q] = so.iperm[(size_t)(m0 + q) * N + i];
        cf[q] = (SUM && d.coef) ? d.coef[i] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (m0 + q < nm) {
        const T* src = k[q] < so.nC ? so.xc : (k[q] < so.nS ? so.xf : so.xd);
        x[q] = (double)src[k[q]];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (m0 + q < nm) {
        const SegOut d = tab[m0 + q];
        z[(size_t)d.seg * N + i] = x[q];
        if (SUM && d.coef) s = s + cf[q] * x[q];
      }
    }
  }
  if (SUM) sT[i] = (T)s;
}

// out = (T)(a - coef o w)   (coef may be null)
template <typename T, typename W>
__global__ void k_single_in(int N, const double* __restrict__ a, const double* __restrict__ coef,
                            const W* __restrict__ w, T* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double v = a ? a[i] : 0.0;
  if (coef) v = a ? v - coef[i] * (double)w[i] : coef[i] * (double)w[i];
  out[i] = (T)v;
}

// z = p - q  (q may be null)
template <typename T>
__global__ void k_sub_out(int N, const T* __restrict__ p, const T* __restrict__ q,
                          double* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  z[i] = q ? (double)p[i] - (double)q[i] : (double)p[i];
}

// E input after independent solves: out = (T)((r - coef o w) - s)  (coef may be null)
template <typename T>
__global__ void k_lower_E_in(int N, const double* __restrict__ r, const double* __restrict__ coef,
                             const T* __restrict__ w, const T* __restrict__ s, T* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double v = r[i];
  if (coef) v = v - coef[i] * (double)w[i];
  v = v - (double)s[i];
  out[i] = (T)v;
}
// One Jacobi iteration (option #1 of Section 3.4) for member blockIdx.y:
// x_out = x_in + (b - A x_in) / d, and x_out = b / d for the first from zero.
template <typename T, bool FIRST>
__global__ void k_jacobi(int N, const JacMember* __restrict__ tab, const T* __restrict__ b,
                         const T* __restrict__ xin, T* __restrict__ xout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const JacMember J = tab[blockIdx.y];
  const size_t off = (size_t)blockIdx.y * N;
  double r = (double)b[off + i];
  if (FIRST) {
    xout[off + i] = (T)(r / J.d[i]);
    return;
  }
  const T* __restrict__ x = xin + off;
  for (int e = J.rp[i]; e < J.rp[i + 1]; ++e) r = r - J.v[e] * (double)x[J.ci[e]];
  xout[off + i] = (T)((double)x[i] + r / J.d[i]);
}
// Definition 1 count: rows with -d_k <= theta a_k
__global__ void k_weak_count(int n, const double* __restrict__ d, const double* __restrict__ a,
                             double theta, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool hit = i < n && -d[i] <= theta * a[i];
  const unsigned long long m = __ballot(hit);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(cnt, (int)__popcll(m));
}
// Definition 2 count: rows with sum_j a_kj < theta a_kk, the sum taken left
// to right in stored (ascending column) order
__global__ void k_wd_count(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, double theta, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool hit = false;
  if (i < n) {
    double s = 0.0, dg = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      s = s + v[e];
      if (ci[e] == i) dg = v[e];
    }
    hit = s < theta * dg;
  }
  const unsigned long long m = __ballot(hit);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(cnt, (int)__popcll(m));
}
// out = (T)(coef o w)
template <typename T>
__global__ void k_coef_mul(int N, const double* __restrict__ coef, const T* __restrict__ w,
                           T* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[i] = (T)(coef[i] * (double)w[i]);
}
// out = (T)(q + coef o t); out may alias q
template <typename T>
__global__ void k_add_coef(int N, const T* q, const double* __restrict__ coef,
                           const T* __restrict__ t, T* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[i] = (T)((double)q[i] + coef[i] * (double)t[i]);
}
// Sum over a 256-thread workgroup; result valid in thread 0.
__device__ __forceinline__ double member_sum256(double v, double* lds /*[4]*/) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
  return r;
}
// Option #3 pieces, member m = blockIdx.y of member-major vectors of N.
// part[m * nb + block] = sum of x_m^2 over the block's grid-stride rows
template <typename T>
__global__ void __launch_bounds__(256) k_member_sq(int N, const T* __restrict__ x,
                                                   double* __restrict__ part, int nb) {
  __shared__ double lds[4];
  const size_t off = (size_t)blockIdx.y * N;
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += nb * 256) {
    const double v = (double)x[off + i];
    s = s + v * v;
  }
  s = member_sum256(s, lds);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * nb + blockIdx.x] = s;
}
// r_m = b_m - A_m z_m (FP64 arithmetic) and its squared norm, active members only
template <typename T>
__global__ void __launch_bounds__(256) k_member_resid(int N, const JacMember* __restrict__ tab,
                                                      const int* __restrict__ active,
                                                      const T* __restrict__ b,
                                                      const T* __restrict__ z, T* __restrict__ r,
                                                      double* __restrict__ part, int nb) {
  __shared__ double lds[4];
  const int m = blockIdx.y;
  if (!active[m]) {  // uniform over the workgroup
    if (threadIdx.x == 0) part[(size_t)m * nb + blockIdx.x] = 0.0;
    return;
  }
  const JacMember A = tab[m];
  const size_t off = (size_t)m * N;
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += nb * 256) {
    double v = (double)b[off + i];
    for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) v = v - A.v[e] * (double)z[off + A.ci[e]];
    r[off + i] = (T)v;
    s = s + v * v;
  }
  s = member_sum256(s, lds);
  if (threadIdx.x == 0) part[(size_t)m * nb + blockIdx.x] = s;
}
// sums[m] = sum_k part[m * nb + k] in a fixed order
__global__ void __launch_bounds__(256) k_member_final(int nb, const double* __restrict__ part,
                                                      double* __restrict__ sums) {
  __shared__ double lds[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) s = s + part[(size_t)blockIdx.x * nb + k];
  s = member_sum256(s, lds);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}
// z_m += t_m for active members
template <typename T>
__global__ void k_member_axpy(int N, const int* __restrict__ active, const T* __restrict__ t,
                              T* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N || !active[blockIdx.y]) return;
  const size_t k = (size_t)blockIdx.y * N + i;
  z[k] = z[k] + t[k];
}
// PCTL restriction of the block residual: rc = r_E + sum_g p_g o r_g + p_I o r_I
template <typename T>
__global__ void k_pctl_restrict(int G, int N, const double* __restrict__ p,
                                const double* __restrict__ res, T* __restrict__ rc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = res[(size_t)G * N + i];
  for (int g = 0; g < G; ++g) s = s + p[(size_t)g * N + i] * res[(size_t)g * N + i];
  s = s + p[(size_t)G * N + i] * res[(size_t)(G + 1) * N + i];
  rc[i] = (T)s;
}
// PCTL coarse correction: w += P w_c
template <typename T>
__global__ void k_pctl_correct(int G, int N, const double* __restrict__ p, const T* __restrict__ wc,
                               double* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double c = (double)wc[i];
  z[(size_t)G * N + i] = z[(size_t)G * N + i] + c;
  for (int g = 0; g < G; ++g) z[(size_t)g * N + i] = z[(size_t)g * N + i] + p[(size_t)g * N + i] * c;
  z[(size_t)(G + 1) * N + i] = z[(size_t)(G + 1) * N + i] + p[(size_t)G * N + i] * c;
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
// a_ii <- a_ii - (d1_i d2_i) / dd_i on the stored diagonal
__global__ void k_hat_update(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                             double* __restrict__ v, const double* __restrict__ d1,
                             const double* __restrict__ d2, const double* __restrict__ dd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] == i) {
      const double t = (d1[i] * d2[i]) / dd[i];
      v[e] = v[e] - t;
    }
}

__global__ void k_get_diag(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] == i) x = v[e];
  d[i] = x;
}

// eq. 3.1 on the shared pattern
__global__ void k_pctl_coarse(int G, int N, BlockSysDev S, const double* __restrict__ p,
                              double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const BlockCsr E = S.blk[G];
  const double* pI = p + (size_t)G * N;
  for (int e = E.rp[i]; e < E.rp[i + 1]; ++e) {
    const int j = E.ci[e];
    double acc = E.v[e];
    for (int g = 0; g < G; ++g) {
      const double* pg = p + (size_t)g * N;
      acc = acc + (pg[i] * S.blk[g].v[e]) * pg[j];
    }
    acc = acc + (pI[i] * S.blk[G + 1].v[e]) * pI[j];
    if (j == i) {
      for (int g = 0; g < G; ++g) {
        const double pg = p[(size_t)g * N + i];
        acc = acc + S.d_Eg[(size_t)g * N + i] * pg;
        acc = acc + pg * S.d_gE[(size_t)g * N + i];
      }
      acc = acc + S.d_EI[i] * pI[i];
      acc = acc + pI[i] * S.d_IE[i];
    }
    out[e] = acc;
  }
}

__global__ void k_pattern_diff(int n, int nnz, const int* __restrict__ rp0,
                               const int* __restrict__ ci0, const int* __restrict__ rp1,
                               const int* __restrict__ ci1, int* __restrict__ diff) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= n && rp0[t] != rp1[t]) diff[0] = 1;
  if (t < nnz && ci0[t] != ci1[t]) diff[0] = 1;
}

__global__ void k_neg(int n, const double* __restrict__ a, double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = -a[i];
}

template <typename T>
void jacobi_run(Ctx* c, int N, const JacMember* tab, int nm, int sweeps, double nnz, const T* b,
                T* x, T* tmp) {
  if (nm <= 0 || N <= 0) return;
  const dim3 grid(cdiv(N, 256), nm);
  // first sweep: b, d, x; later ones: the matrix, the row pointers, b, d, x in and out
  const double first = (double)nm * N * (2.0 * sizeof(T) + 8.0);
  const double later = 12.0 * nnz + (double)nm * N * (4.0 + 3.0 * sizeof(T) + 8.0);
  ProfScope ps(c, KC_SMOOTH_L0, first + (sweeps - 1) * later, ksym(c, "k_jacobi", {type_name<T>()}));
  // sweep s writes x when (sweeps - s) is even, so the last one lands in x
  const T* src = nullptr;
  for (int s = 1; s <= sweeps; ++s) {
    T* dst = ((sweeps - s) % 2 == 0) ? x : tmp;
    if (s == 1)
      hipLaunchKernelGGL((k_jacobi<T, true>), grid, dim3(256), 0, c->stream, N, tab, b,
                         (const T*)nullptr, dst);
    else
      hipLaunchKernelGGL((k_jacobi<T, false>), grid, dim3(256), 0, c->stream, N, tab, b, src, dst);
    MGD_CHECK_LAUNCH();
    src = dst;
  }
}
template void jacobi_run<double>(Ctx*, int, const JacMember*, int, int, double, const double*,
                                 double*, double*);
template void jacobi_run<float>(Ctx*, int, const JacMember*, int, int, double, const float*, float*,
                                float*);

template <typename T>
void Group<T>::run(Ctx* c, int N) {
  if (n_amg > 0) {
    if (batched) {
      batched->apply(c, in.get(), out.get(), cycles);
    } else {
      for (size_t m = 0; m < seq.size(); ++m)
        seq[m]->apply(c, in.get() + m * (size_t)N, out.get() + m * (size_t)N, cycles);
    }
  }
  const int nj = (int)roles.size() - n_amg;
  if (nj > 0)
    jacobi_run<T>(c, N, jac_tab.get(), nj, jac_sweeps, jac_nnz, in.get() + (size_t)n_amg * N,
                  out.get() + (size_t)n_amg * N, jac_tmp.get());
}
template struct Group<double>;
template struct Group<float>;

}  // namespace mgd

// ===========================================================================
// block_precond
// ===========================================================================
block_precond::~block_precond() {
  for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
  for (auto& kv : step_graphs) hipGraphExecDestroy(kv.second);
  if (aux) hipStreamDestroy(aux);
  if (ev_in) hipEventDestroy(ev_in);
  if (ev_out) hipEventDestroy(ev_out);
  if (ovl_stream) hipStreamDestroy(ovl_stream);
  if (ovl_fork) hipEventDestroy(ovl_fork);
  if (ovl_join) hipEventDestroy(ovl_join);
  if (fs_fork) hipEventDestroy(fs_fork);
  if (fs_join) hipEventDestroy(fs_join);
}

static void make_hierarchy(block_precond* bp, int role, Csr<double>&& M) {
  auto h = std::make_unique<amg_hierarchy>();
  h->ctx = bp->ctx;
  h->prm = bp->prm.amg;
  h->n = M.n_rows;
  auto t0 = std::chrono::steady_clock::now();
  amg_build(bp->ctx, std::move(M), h->prm, h->H);
  h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if ((int)bp->hier.size() <= role) bp->hier.resize(role + 1);
  bp->hier[role] = std::move(h);
}

static void diag_of(Ctx* c, const Csr<double>& A, double* d) {
  hipLaunchKernelGGL(k_get_diag, dim3(cdiv(A.n_rows, 256)), dim3(256), 0, c->stream, A.n_rows,
                     A.rp.get(), A.ci.get(), A.v.get(), d);
  MGD_CHECK_LAUNCH();
}

static Csr<double> hat(Ctx* c, const Csr<double>& A, const double* d1, const double* d2,
                       const double* dd) {
  Csr<double> B;
  csr_copy(c, A, B);
  hipLaunchKernelGGL(k_hat_update, dim3(cdiv(B.n_rows, 256)), dim3(256), 0, c->stream, B.n_rows,
                     B.rp.get(), B.ci.get(), B.v.get(), d1, d2, dd);
  MGD_CHECK_LAUNCH();
  return B;
}

// Option #3: V-cycles on the hierarchy until ||rhs - A z|| < tol ||rhs||.
static int solve_to_tol(block_precond* bp, amg_hierarchy* h, const double* rhs, double* z,
                        double tol, int maxc) {
  Ctx* c = bp->ctx;
  const int n = h->n;
  Union<double>* U = h->union64();
  DBuf<double> r(c, n), t(c, n), nrm(c, 2);
  RedWork rw;
  fill<double>(c, z, 0.0, n);
  copy_d2d(c, r.get(), rhs, n);
  dot_dev(c, rw, rhs, rhs, n, nrm.get());
  const double nb = std::sqrt(read1(c, nrm.get()));
  if (nb == 0.0) return 0;
  const CsrView<double> A0 = view(h->H.levels[0].A);
  const int tpr = default_tpr((double)A0.nnz / std::max(1, A0.n_rows));
  int k = 0;
  while (k < maxc) {
    U->apply(c, r.get(), t.get(), 1);
    axpy(c, z, t.get(), 1.0, n);
    ++k;
    spmv(c, A0, z, r.get(), tpr, KC_SPMV);
    rsub(c, rhs, r.get(), n);
    dot_dev(c, rw, r.get(), r.get(), n, nrm.get() + 1);
    if (std::sqrt(read1(c, nrm.get() + 1)) < tol * nb) break;
  }
  return k;
}

// The inverses Section 4 solves to a relative tolerance: the hatted matrices
// of the Schur preconditioners and PCTL's block relaxations.
static bool tolerance_role(int kind, int role, int G, bool option4) {
  if (option4 && ((kind == MGD_PC_SCHUR2 && role == G + 1) || (kind == MGD_PC_SCHUR1 && role == G)))
    return false;  // option #4 iterates on the original block instead
  if (role < G) return kind == MGD_PC_SCHUR1 || kind == MGD_PC_SCHUR2 ||
                       kind == MGD_PC_SCHUR2_LOWER || kind == MGD_PC_PCTL;
  if (role == G) return kind == MGD_PC_SCHUR1 || kind == MGD_PC_PCTL;
  if (role == G + 1)
    return kind == MGD_PC_SCHUR2 || kind == MGD_PC_SCHUR2_LOWER || kind == MGD_PC_PCTL;
  return false;
}

template <typename T>
static std::unique_ptr<TolSolve<T>> make_tol(block_precond* bp, const std::vector<int>& roles) {
  Ctx* c = bp->ctx;
  const int N = bp->N, nm = (int)roles.size();
  auto S = std::make_unique<TolSolve<T>>();
  S->roles = roles;
  std::vector<JacMember> tab;
  for (int r : roles) {
    const Csr<double>& A = bp->hier[r]->H.levels[0].A;
    tab.push_back({A.rp.get(), A.ci.get(), A.v.get(), nullptr});
    S->nnz += (double)A.nnz;
  }
  S->mats.alloc(c, (size_t)nm);
  copy_h2d(c, S->mats.get(), tab.data(), (size_t)nm);
  S->r.alloc(c, (size_t)nm * N);
  S->t.alloc(c, (size_t)nm * N);
  S->active.alloc(c, (size_t)nm);
  S->nb = (int)std::min<long long>(cdiv(N, 256), 128);
  S->part.alloc(c, (size_t)nm * S->nb);
  S->sums.alloc(c, (size_t)nm);
  return S;
}

// Option #3 over the members of S: z = 0, r = b; then V-cycles z += V(r),
// r = b - A z, a member leaving once ||r|| < inner_tol ||b|| (members with
// b = 0 take no cycle).  `vcycle` runs one V-cycle on all members at once.
template <typename T, typename V>
static void tol_run(block_precond* bp, TolSolve<T>& S, const T* b, T* z, V&& vcycle) {
  Ctx* c = bp->ctx;
  const int N = bp->N, nm = (int)S.roles.size();
  const size_t nN = (size_t)nm * N;
  const double tol = bp->prm.inner_tol;
  const int maxc = bp->prm.inner_maxcycles;
  const dim3 gr(S.nb, nm), g1(cdiv(N, 256), nm), b256(256);
  hipLaunchKernelGGL(k_member_sq<T>, gr, b256, 0, c->stream, N, b, S.part.get(), S.nb);
  hipLaunchKernelGGL(k_member_final, dim3(nm), b256, 0, c->stream, S.nb,
                     (const double*)S.part.get(), S.sums.get());
  MGD_CHECK_LAUNCH();
  std::vector<double> bn2((size_t)nm), rn2((size_t)nm);
  copy_d2h(c, bn2.data(), S.sums.get(), (size_t)nm);
  std::vector<int> act((size_t)nm), cyc((size_t)nm, 0);
  int n_act = 0;
  for (int m = 0; m < nm; ++m) {
    act[m] = bn2[m] > 0.0 ? 1 : 0;
    n_act += act[m];
  }
  fill<T>(c, z, (T)0, nN);
  cast_copy<T, T>(c, S.r.get(), b, nN, KC_VEC);
  copy_h2d(c, S.active.get(), act.data(), (size_t)nm);
  for (int k = 1; k <= maxc && n_act > 0; ++k) {
    vcycle((const T*)S.r.get(), S.t.get());
    {
      ProfScope ps(c, KC_VEC, 12.0 * S.nnz + (double)nN * (4.0 + 4.0 * sizeof(T)),
                   ksym(c, "k_member_resid", {type_name<T>()}));
      hipLaunchKernelGGL(k_member_axpy<T>, g1, b256, 0, c->stream, N, (const int*)S.active.get(),
                         (const T*)S.t.get(), z);
      hipLaunchKernelGGL(k_member_resid<T>, gr, b256, 0, c->stream, N,
                         (const JacMember*)S.mats.get(), (const int*)S.active.get(), b,
                         (const T*)z, S.r.get(), S.part.get(), S.nb);
      hipLaunchKernelGGL(k_member_final, dim3(nm), b256, 0, c->stream, S.nb,
                         (const double*)S.part.get(), S.sums.get());
      MGD_CHECK_LAUNCH();
    }
    copy_d2h(c, rn2.data(), S.sums.get(), (size_t)nm);
    bool changed = false;
    for (int m = 0; m < nm; ++m) {
      if (!act[m]) continue;
      if (std::sqrt(rn2[m]) < tol * std::sqrt(bn2[m]) || k == maxc) {
        act[m] = 0;
        cyc[m] = k;
        --n_act;
        changed = true;
      }
    }
    if (changed && n_act > 0) copy_h2d(c, S.active.get(), act.data(), (size_t)nm);
  }
  for (int m = 0; m < nm; ++m) bp->inner_cycles[S.roles[m]] = cyc[m];
}

template <typename T>
static void build_exec(block_precond* bp, std::unique_ptr<PcExec<T>>& X) {
  Ctx* c = bp->ctx;
  const int G = bp->G, N = bp->N;
  const int kind = bp->prm.kind;
  X = std::make_unique<PcExec<T>>();
  if (kind == MGD_PC_IDENTITY) return;
  // every single-hierarchy union the apply uses is built here, so that an
  // apply (possibly under graph capture) never allocates
  std::vector<int> singles;
  if (kind == MGD_PC_AMG_MONO) singles = {0};
  if (kind == MGD_PC_SCHUR2 || kind == MGD_PC_SCHUR2_LOWER) singles = {G};
  if (kind == MGD_PC_SCHUR2 && bp->prm.option4_steps > 0) singles = {G, G + 1};
  if (kind == MGD_PC_PCTL) singles = {G, G + 2};
  if (kind == MGD_PC_SCHUR1) singles = {G, G + 1};
  X->jac_one.resize(G + 3);
  X->tol_one.resize(G + 3);
  const bool inner = bp->prm.inner_tol > 0;
  for (int r : singles) {
    if (inner && bp->tol_role[r] && !bp->jacobi[r]) X->tol_one[r] = make_tol<T>(bp, {r});
    if (bp->jacobi[r]) {
      const Csr<double>& A = bp->hier[r]->H.levels[0].A;
      JacMember jm{A.rp.get(), A.ci.get(), A.v.get(), bp->jac_diag[r].get()};
      X->jac_one[r].alloc(c, 1);
      copy_h2d(c, X->jac_one[r].get(), &jm, 1);
      if (X->jac_tmp1.n < (size_t)N) X->jac_tmp1.alloc(c, (size_t)std::max(N, 1));
    } else {
      union_of<T>(bp->hier[r].get());
    }
  }
  const size_t n1 = (size_t)std::max(N, 1);
  X->a_out.alloc(c, (kind == MGD_PC_AMG_MONO) ? (size_t)(G + 2) * N : n1);
  X->a_in.alloc(c, (kind == MGD_PC_AMG_MONO) ? (size_t)(G + 2) * N : n1);
  X->b_in.alloc(c, n1);
  X->b_out.alloc(c, n1);
  X->s.alloc(c, n1);
  if (kind == MGD_PC_PCTL) X->res.alloc(c, (size_t)(G + 2) * N);
  if (bp->prm.option4_steps > 0) {
    X->o4_w.alloc(c, n1);
    X->o4_s.alloc(c, n1);
    X->o4_t.alloc(c, n1);
    X->o4_u.alloc(c, n1);
  }
  {
    const SegIn st[2] = {{G, nullptr}, {G + 1, nullptr}};
    X->seg_tab.alloc(c, 2);
    copy_h2d(c, X->seg_tab.get(), st, 2);
  }
  if (kind == MGD_PC_AMG_MONO) return;
  // group membership
  std::vector<SegIn> tin;
  std::vector<SegOut> tout;
  std::vector<int> roles;
  const double* dgE = bp->d_gE.get();
  const double* dEg = bp->d_Eg.get();
  // a neglected coupling (adaptive strategy) contributes no term at all
  const bool adp = bp->prm.adaptive != 0;
  auto gE = [&](int g) { return (adp && bp->weak_gE[g]) ? nullptr : dgE + (size_t)g * N; };
  auto Eg = [&](int g) { return (adp && bp->weak_Eg[g]) ? nullptr : dEg + (size_t)g * N; };
  const double* IE = (adp && bp->weak_IE) ? nullptr : bp->d_IE.get();
  const double* EI = (adp && bp->weak_EI) ? nullptr : bp->d_EI.get();
  if (kind == MGD_PC_BLOCK_DIAG) {
    for (int a = 0; a < G + 2; ++a) {
      roles.push_back(a);
      tin.push_back({a, nullptr});
      tout.push_back({a, nullptr});
    }
  } else if (kind == MGD_PC_SCHUR1) {
    for (int g = 0; g < G; ++g) {
      roles.push_back(g);
      tin.push_back({g, gE(g)});
      tout.push_back({g, Eg(g)});
    }
  } else {  // SCHUR2, SCHUR2_LOWER, PCTL: groups and I after E
    const bool sum = kind == MGD_PC_SCHUR2;
    for (int g = 0; g < G; ++g) {
      roles.push_back(g);
      tin.push_back({g, gE(g)});
      tout.push_back({g, sum ? Eg(g) : nullptr});
    }
    if (!(kind == MGD_PC_SCHUR2 && bp->prm.option4_steps > 0)) {  // else I by option #4
      roles.push_back(G + 1);
      tin.push_back({G + 1, IE});
      tout.push_back({G + 1, sum ? EI : nullptr});
    }
  }
  // V-cycle members first, Jacobi members (option #1) after them
  {
    std::vector<size_t> order(roles.size());
    for (size_t m = 0; m < order.size(); ++m) order[m] = m;
    std::stable_partition(order.begin(), order.end(),
                          [&](size_t m) { return !bp->jacobi[roles[m]]; });
    std::vector<int> r2;
    std::vector<SegIn> i2;
    std::vector<SegOut> o2;
    for (size_t m : order) {
      r2.push_back(roles[m]);
      i2.push_back(tin[m]);
      o2.push_back(tout[m]);
    }
    roles.swap(r2);
    tin.swap(i2);
    tout.swap(o2);
  }
  Group<T>& grp = X->grp;
  grp.roles = roles;
  int n_amg = 0;
  for (int r : roles) n_amg += bp->jacobi[r] ? 0 : 1;
  grp.n_amg = n_amg;
  grp.cycles = n_amg > 0 ? bp->cycles[roles[0]] : 1;
  bool uniform = true;
  for (int m = 0; m < n_amg; ++m) uniform = uniform && bp->cycles[roles[m]] == grp.cycles;
  const size_t nm = roles.size();
  grp.in.alloc(c, nm * N);
  grp.out.alloc(c, nm * N);
  grp.in_tab.alloc(c, nm);
  grp.out_tab.alloc(c, nm);
  copy_h2d(c, grp.in_tab.get(), tin.data(), nm);
  copy_h2d(c, grp.out_tab.get(), tout.data(), nm);
  if (bp->prm.batched && uniform && n_amg > 1) {
    std::vector<const SetupHierarchy*> hs;
    for (int m = 0; m < n_amg; ++m) hs.push_back(&bp->hier[roles[m]]->H);
    grp.batched = build_union<T>(c, hs, bp->prm.amg.n_pre, bp->prm.amg.n_post, bp->prm.amg.autotune,
                                bp->prm.amg.smoother);
  } else {
    for (int m = 0; m < n_amg; ++m) grp.seq.push_back(union_of<T>(bp->hier[roles[m]].get()));
    if (!uniform) {
      // members with different cycle counts run one by one with their own count
      grp.cycles = -1;
    }
  }
  if (inner && n_amg > 0) {
    bool all_tol = true;
    for (int m = 0; m < n_amg; ++m) all_tol = all_tol && bp->tol_role[roles[m]];
    MGD_REQUIRE(all_tol, "internal: a batched step mixes fixed-count and tolerance inverses");
    grp.tol = make_tol<T>(bp, std::vector<int>(roles.begin(), roles.begin() + n_amg));
  }
  const int nj = (int)nm - n_amg;
  if (nj > 0) {
    std::vector<JacMember> jt;
    for (size_t m = n_amg; m < nm; ++m) {
      const Csr<double>& A = bp->hier[roles[m]]->H.levels[0].A;
      jt.push_back({A.rp.get(), A.ci.get(), A.v.get(), bp->jac_diag[roles[m]].get()});
      grp.jac_nnz += (double)A.nnz;
    }
    grp.jac_tab.alloc(c, (size_t)nj);
    copy_h2d(c, grp.jac_tab.get(), jt.data(), (size_t)nj);
    grp.jac_sweeps = bp->prm.jacobi_sweeps;
    grp.jac_tmp.alloc(c, (size_t)nj * N);
  }
}

template <typename T>
static const T* as_input(Ctx* c, const double* src, DBuf<T>& tmp, int N) {
  if constexpr (std::is_same<T, double>::value) {
    (void)c;
    (void)tmp;
    (void)N;
    return src;
  } else {
    cast_copy<float, double>(c, tmp.get(), src, (size_t)N, KC_VEC);
    return tmp.get();
  }
}

template <typename T>
static void run_group(block_precond* bp, Group<T>& grp) {
  Ctx* c = bp->ctx;
  const int N = bp->N;
  if (grp.tol) {
    // option #3 on the V-cycle members (one V-cycle per inner step), then
    // the Jacobi members
    tol_run<T>(bp, *grp.tol, grp.in.get(), grp.out.get(), [&](const T* rin, T* tout) {
      if (grp.batched) {
        grp.batched->apply(c, rin, tout, 1);
      } else {
        for (size_t m = 0; m < grp.seq.size(); ++m)
          grp.seq[m]->apply(c, rin + m * (size_t)N, tout + m * (size_t)N, 1);
      }
    });
    const int nj = (int)grp.roles.size() - grp.n_amg;
    if (nj > 0)
      jacobi_run<T>(c, N, grp.jac_tab.get(), nj, grp.jac_sweeps, grp.jac_nnz,
                    grp.in.get() + (size_t)grp.n_amg * N, grp.out.get() + (size_t)grp.n_amg * N,
                    grp.jac_tmp.get());
    return;
  }
  if (grp.cycles >= 0) {
    grp.run(c, N);
    return;
  }
  for (size_t m = 0; m < grp.seq.size(); ++m)
    grp.seq[m]->apply(c, grp.in.get() + m * (size_t)N, grp.out.get() + m * (size_t)N,
                      bp->cycles[grp.roles[m]]);
  const int nj = (int)grp.roles.size() - grp.n_amg;
  if (nj > 0)
    jacobi_run<T>(c, N, grp.jac_tab.get(), nj, grp.jac_sweeps, grp.jac_nnz,
                  grp.in.get() + (size_t)grp.n_amg * N, grp.out.get() + (size_t)grp.n_amg * N,
                  grp.jac_tmp.get());
}

template <typename T>
static void apply_impl(block_precond* bp, PcExec<T>& X, const double* r, double* z) {
  Ctx* c = bp->ctx;
  const int G = bp->G, N = bp->N, kind = bp->prm.kind;
  const size_t nN = (size_t)N;
  const dim3 g1(cdiv(N, 256)), b1(256);
  int ninv = 0, nmv = 0;
  auto U = [&](int role) { return union_of<T>(bp->hier[role].get()); };
  const bool adaptive = bp->prm.adaptive != 0;
  // one scalar inverse: V-cycles, or Jacobi iterations (option #1)
  auto inv = [&](int role, const T* in, T* out) {
    if (X.tol_one[role])
      tol_run<T>(bp, *X.tol_one[role], in, out,
                 [&](const T* rin, T* tout) { U(role)->apply(c, rin, tout, 1); });
    else if (bp->jacobi[role])
      jacobi_run<T>(c, N, X.jac_one[role].get(), 1, bp->prm.jacobi_sweeps,
                    (double)bp->hier[role]->H.levels[0].A.nnz, in, out, X.jac_tmp1.get());
    else
      U(role)->apply(c, in, out, bp->cycles[role]);
  };
  // option #4 (Schur2: S_I, Schur1: C_E): w = A_o^{-1} q, then
  // w <- A_o^{-1}(q + D_oi A_i^{-1}(D_io w)) for the remaining steps
  const int steps4 = bp->prm.option4_steps;
  int extra_inv = 0;
  auto opt4 = [&](const T* q, T* w) {
    const bool s2 = kind == MGD_PC_SCHUR2;
    const int outer = s2 ? G + 1 : G, inner = s2 ? G : G + 1;
    const double* d_out = s2 ? bp->d_IE.get() : bp->d_EI.get();
    const double* d_in = s2 ? bp->d_EI.get() : bp->d_IE.get();
    inv(outer, q, w);
    for (int k = 1; k < steps4; ++k) {
      hipLaunchKernelGGL(k_coef_mul<T>, g1, b1, 0, c->stream, N, d_in, (const T*)w, X.o4_s.get());
      MGD_CHECK_LAUNCH();
      inv(inner, X.o4_s.get(), X.o4_t.get());
      hipLaunchKernelGGL(k_add_coef<T>, g1, b1, 0, c->stream, N, q, d_out,
                         (const T*)X.o4_t.get(), X.o4_u.get());
      MGD_CHECK_LAUNCH();
      inv(outer, X.o4_u.get(), w);
    }
    extra_inv += 2 * steps4 - 2;
  };
  // out = inverse of role applied to segment seg (E or I) of r; in FP32 a
  // plain single V-cycle takes the segment in its entry kernel (the cast and
  // the cycle's arithmetic unchanged)
  auto inv_seg = [&](int role, int seg, T* out) {
    if (std::is_same<T, float>::value && !X.tol_one[role] && !bp->jacobi[role] &&
        bp->cycles[role] == 1) {
      U(role)->apply_seg(c, N, X.seg_tab.get() + (seg - G), r, nullptr, out);
      return;
    }
    inv(role, as_input<T>(c, r + (size_t)seg * N, X.a_in, N), out);
  };
  // the Schur complement inverse of the kind: option #4 when asked for
  auto cinv = [&](int role, const T* in, T* out) {
    if (steps4 > 0 && ((kind == MGD_PC_SCHUR2 && role == G + 1) ||
                       (kind == MGD_PC_SCHUR1 && role == G)))
      opt4(in, out);
    else
      inv(role, in, out);
  };
  Group<T>& grp = X.grp;
  const int nm = (int)grp.roles.size();
  auto group_in = [&](const T* w) {
    ProfScope ps(c, KC_VEC, (double)nm * N * (8 + 8 + sizeof(T)) + N * sizeof(T));
    hipLaunchKernelGGL(k_group_in<T>, dim3(cdiv(N, 256), nm), b1, 0, c->stream, N,
                       (const SegIn*)grp.in_tab.get(), r, w, grp.in.get());
    MGD_CHECK_LAUNCH();
  };
  // group_in, then the group's inverses; a batched group of V-cycle members
  // with one cycle each forms its inputs in the union's entry kernel instead,
  // and (CF-l1-Jacobi, MGD_STORED_OUT not 0) leaves its result in stored
  // order for group_out to read
  bool grp_stored = false;
  auto group_solve = [&](const T* w) {
    grp_stored = false;
    if (!grp.tol && grp.cycles == 1 && grp.batched && grp.n_amg == nm) {
      const char* so = std::getenv("MGD_STORED_OUT");
      grp_stored = !grp.batched->gs && grp.batched->tail_from != 0 && !(so && so[0] == '0');
      grp.batched->apply_seg(c, N, (const SegIn*)grp.in_tab.get(), r, w,
                             grp_stored ? nullptr : grp.out.get());
      return;
    }
    group_in(w);
    run_group(bp, grp);
  };
  auto group_out = [&](bool sum, T* sT) {
    if (grp_stored) {
      ProfScope ps(c, KC_VEC, (double)nm * N * (4 + sizeof(T) + 8 + (sum ? 8 : 0)),
                   ksym(c, "k_group_out_st", {type_name<T>(), sum ? "true" : "false"}));
      const StoredOut<T> so = grp.batched->stored_out();
      if (sum)
        hipLaunchKernelGGL((k_group_out_st<T, true>), g1, b1, 0, c->stream, N, nm,
                           (const SegOut*)grp.out_tab.get(), so, z, sT);
      else
        hipLaunchKernelGGL((k_group_out_st<T, false>), g1, b1, 0, c->stream, N, nm,
                           (const SegOut*)grp.out_tab.get(), so, z, sT);
      MGD_CHECK_LAUNCH();
      return;
    }
    ProfScope ps(c, KC_VEC, (double)nm * N * (sizeof(T) + 8 + (sum ? 8 : 0)),
                 ksym(c, "k_group_out", {type_name<T>(), sum ? "true" : "false"}));
    if (sum)
      hipLaunchKernelGGL((k_group_out<T, true>), g1, b1, 0, c->stream, N, nm,
                         (const SegOut*)grp.out_tab.get(), (const T*)grp.out.get(), z, sT);
    else
      hipLaunchKernelGGL((k_group_out<T, false>), g1, b1, 0, c->stream, N, nm,
                         (const SegOut*)grp.out_tab.get(), (const T*)grp.out.get(), z, sT);
    MGD_CHECK_LAUNCH();
  };
  switch (kind) {
    case MGD_PC_IDENTITY:
      cast_copy<double, double>(c, z, r, (size_t)(G + 2) * N, KC_VEC);
      break;
    case MGD_PC_AMG_MONO: {
      const size_t n = (size_t)(G + 2) * N;
      if constexpr (std::is_same<T, double>::value) {
        U(0)->apply(c, r, z, bp->cycles[0]);
      } else {
        cast_copy<float, double>(c, X.a_in.get(), r, n, KC_VEC);
        U(0)->apply(c, X.a_in.get(), X.a_out.get(), bp->cycles[0]);
        cast_copy<double, float>(c, z, X.a_out.get(), n, KC_VEC);
      }
      ninv = 1;
      break;
    }
    case MGD_PC_BLOCK_DIAG:
      group_solve(nullptr);
      group_out(false, nullptr);
      ninv = G + 2;
      break;
    case MGD_PC_SCHUR2:
    case MGD_PC_SCHUR2_LOWER:
    case MGD_PC_PCTL: {
      const bool i_apart = kind == MGD_PC_SCHUR2 && steps4 > 0;  // S_I by option #4
      const double* dIE = (adaptive && bp->weak_IE) ? nullptr : bp->d_IE.get();
      const double* dEI = (adaptive && bp->weak_EI) ? nullptr : bp->d_EI.get();
      // w_I = S_I^{-1}(r_I - D_IE w) by option #4 (w null: r_I), into z; then
      // sT += D_EI w_I when sT is given
      auto i_step = [&](const T* w, T* sT) {
        hipLaunchKernelGGL((k_single_in<T, T>), g1, b1, 0, c->stream, N, r + (size_t)(G + 1) * N,
                           w ? dIE : (const double*)nullptr, w, X.b_out.get());
        MGD_CHECK_LAUNCH();
        cinv(G + 1, X.b_out.get(), X.o4_w.get());
        hipLaunchKernelGGL(k_sub_out<T>, g1, b1, 0, c->stream, N, (const T*)X.o4_w.get(),
                           (const T*)nullptr, z + (size_t)(G + 1) * N);
        MGD_CHECK_LAUNCH();
        if (sT && dEI) {
          hipLaunchKernelGGL(k_add_coef<T>, g1, b1, 0, c->stream, N, (const T*)sT, dEI,
                             (const T*)X.o4_w.get(), sT);
          MGD_CHECK_LAUNCH();
        }
      };
      if (adaptive && kind == MGD_PC_SCHUR2 && bp->from_E_weak) {
        // every row block independent of E (block lower triangular):
        // w_a = S^_a^{-1} r_a, then w_E = A_E^{-1}(r_E - sum_a D_Ea w_a)
        group_solve(nullptr);
        group_out(true, X.b_in.get());
        if (i_apart) i_step(nullptr, X.b_in.get());
        hipLaunchKernelGGL(k_lower_E_in<T>, g1, b1, 0, c->stream, N, r + (size_t)G * N,
                           (const double*)nullptr, (const T*)nullptr, (const T*)X.b_in.get(),
                           X.b_out.get());
        MGD_CHECK_LAUNCH();
        inv(G, X.b_out.get(), X.a_out.get());
        hipLaunchKernelGGL(k_sub_out<T>, g1, b1, 0, c->stream, N, (const T*)X.a_out.get(),
                           (const T*)nullptr, z + (size_t)G * N);
        MGD_CHECK_LAUNCH();
        ninv = G + 2 + extra_inv;
        break;
      }
      // step 1: w_E* = A_E^{-1} r_E (or already in X.a_out: first_stage 2)
      if (bp->first_stage != 2) {
        inv_seg(G, G, X.a_out.get());
        if (bp->first_stage == 1) return;
      }
      // step 2: groups and I against r - D_.E w_E*
      group_solve(X.a_out.get());
      ninv = 1 + G + 1;
      const bool e_coupled = !(adaptive && bp->into_E_weak);
      if (kind == MGD_PC_SCHUR2 && e_coupled) {
        // step 3: w_E = w_E* - A_E^{-1}(sum_g D_Eg w_g + D_EI w_I)
        group_out(true, X.b_in.get());
        if (i_apart) i_step(X.a_out.get(), X.b_in.get());
        const bool fork = bp->ovl_S != nullptr;
        if (fork) {  // the part of A z that needs no z_E runs beside the E solve
          MGD_HIP(hipEventRecord(bp->ovl_fork, c->stream));
          MGD_HIP(hipStreamWaitEvent(bp->ovl_stream, bp->ovl_fork, 0));
          block_matvec_split(c, *bp->ovl_S, z, bp->ovl_y, bp->ovl_stream);
          MGD_HIP(hipEventRecord(bp->ovl_join, bp->ovl_stream));
        }
        inv(G, X.b_in.get(), X.b_out.get());
        hipLaunchKernelGGL(k_sub_out<T>, g1, b1, 0, c->stream, N, (const T*)X.a_out.get(),
                           (const T*)X.b_out.get(), z + (size_t)G * N);
        MGD_CHECK_LAUNCH();
        if (fork) {
          MGD_HIP(hipStreamWaitEvent(c->stream, bp->ovl_join, 0));
          bp->ovl_forked = true;
        }
        ninv += 1;
      } else {
        group_out(false, nullptr);
        if (i_apart) i_step(X.a_out.get(), nullptr);
        hipLaunchKernelGGL(k_sub_out<T>, g1, b1, 0, c->stream, N, (const T*)X.a_out.get(),
                           (const T*)nullptr, z + (size_t)G * N);
        MGD_CHECK_LAUNCH();
      }
      ninv += extra_inv;
      if (kind == MGD_PC_PCTL && e_coupled) {
        // coarse-grid correction: A_c w_c = P^T (b - A w); w += P w_c
        block_matvec(c, bp->sys, z, r, X.res.get());
        nmv = G + 2;
        hipLaunchKernelGGL(k_pctl_restrict<T>, g1, b1, 0, c->stream, G, N,
                           (const double*)bp->p.get(), (const double*)X.res.get(), X.b_in.get());
        MGD_CHECK_LAUNCH();
        U(G + 2)->apply(c, X.b_in.get(), X.b_out.get(), bp->cycles[G + 2]);
        hipLaunchKernelGGL(k_pctl_correct<T>, g1, b1, 0, c->stream, G, N,
                           (const double*)bp->p.get(), (const T*)X.b_out.get(), z);
        MGD_CHECK_LAUNCH();
        ninv += 1;
      }
      break;
    }
    case MGD_PC_SCHUR1: {
      const double* dEI = (adaptive && bp->weak_EI) ? nullptr : bp->d_EI.get();
      // 1. w_I* = A_I^{-1} r_I
      inv_seg(G + 1, G + 1, X.a_out.get());
      if (adaptive && bp->groups_from_E_weak) {
        // groups independent of E: w_g = C^_g^{-1} r_g, then one C^_E inverse
        // w_E = C^_E^{-1}((r_E - D_EI w_I*) - sum_g D_Eg w_g)
        group_solve(nullptr);
        group_out(true, X.b_in.get());
        hipLaunchKernelGGL(k_lower_E_in<T>, g1, b1, 0, c->stream, N, r + (size_t)G * N, dEI,
                           (const T*)X.a_out.get(), (const T*)X.b_in.get(), X.b_out.get());
        MGD_CHECK_LAUNCH();
        cinv(G, X.b_out.get(), X.b_in.get());
        hipLaunchKernelGGL(k_sub_out<T>, g1, b1, 0, c->stream, N, (const T*)X.b_in.get(),
                           (const T*)nullptr, z + (size_t)G * N);
        MGD_CHECK_LAUNCH();
        ninv = 1 + G + 1;
      } else {
        // 2. w_E* = C^_E^{-1}(r_E - D_EI w_I*)
        hipLaunchKernelGGL((k_single_in<T, T>), g1, b1, 0, c->stream, N, r + (size_t)G * N, dEI,
                           (const T*)X.a_out.get(), X.b_in.get());
        MGD_CHECK_LAUNCH();
        cinv(G, X.b_in.get(), X.b_out.get());
        // 3. w_g = C^_g^{-1}(r_g - D_gE w_E*)
        group_solve(X.b_out.get());
        ninv = 1 + 1 + G;
        if (adaptive && bp->into_E_weak_groups) {
          group_out(false, nullptr);
          hipLaunchKernelGGL(k_sub_out<T>, g1, b1, 0, c->stream, N, (const T*)X.b_out.get(),
                             (const T*)nullptr, z + (size_t)G * N);
          MGD_CHECK_LAUNCH();
        } else {
          // 4. w_E = w_E* - C^_E^{-1} sum_g D_Eg w_g
          group_out(true, X.b_in.get());
          DBuf<T>& tmp = X.a_in;  // free after step 1 (FP32) / unused (FP64)
          if (tmp.n < nN) tmp.alloc(c, nN);
          cinv(G, X.b_in.get(), tmp.get());
          hipLaunchKernelGGL(k_sub_out<T>, g1, b1, 0, c->stream, N, (const T*)X.b_out.get(),
                             (const T*)tmp.get(), z + (size_t)G * N);
          MGD_CHECK_LAUNCH();
          ninv += 1;
        }
      }
      if (adaptive && bp->weak_IE) {
        hipLaunchKernelGGL(k_sub_out<T>, g1, b1, 0, c->stream, N, (const T*)X.a_out.get(),
                           (const T*)nullptr, z + (size_t)(G + 1) * N);
        MGD_CHECK_LAUNCH();
      } else {
        // 5. w_I = w_I* - A_I^{-1} D_IE w_E
        hipLaunchKernelGGL((k_single_in<T, double>), g1, b1, 0, c->stream, N,
                           (const double*)nullptr, (const double*)bp->d_IE.get(),
                           (const double*)(z + (size_t)G * N), X.b_in.get());
        MGD_CHECK_LAUNCH();
        inv(G + 1, X.b_in.get(), X.b_out.get());
        hipLaunchKernelGGL(k_sub_out<T>, g1, b1, 0, c->stream, N, (const T*)X.a_out.get(),
                           (const T*)X.b_out.get(), z + (size_t)(G + 1) * N);
        MGD_CHECK_LAUNCH();
        ninv += 1;
      }
      ninv += extra_inv;
      break;
    }
    default:
      fail(MGD_EINVAL, "unknown preconditioner kind");
  }
  bp->inverses_last = ninv;
  bp->matvecs_last = nmv;
}

void block_precond_graph_launch(block_precond* bp, const double* r, double* z);

void block_precond_apply_impl(block_precond* bp, const double* r, double* z) {
  if (bp->prm.amg.precision == 1 && bp->prm.kind != MGD_PC_IDENTITY)
    apply_impl<float>(bp, *bp->x32, r, z);
  else
    apply_impl<double>(bp, *bp->x64, r, z);
}

void block_precond_apply_dispatch(block_precond* bp, const double* r, double* z) {
  Ctx* c = bp->ctx;
  if (!bp->prm.use_graph || c->profiling || c->no_alloc || bp->prm.inner_tol > 0) {
    block_precond_apply_impl(bp, r, z);
    return;
  }
  // Capture and replay need a real stream: on the null stream the graph runs
  // on a private non-blocking stream ordered after and before the caller's.
  const hipStream_t user = c->stream;
  if (user == nullptr) {
    if (!bp->aux) {
      MGD_HIP(hipStreamCreateWithFlags(&bp->aux, hipStreamNonBlocking));
      MGD_HIP(hipEventCreateWithFlags(&bp->ev_in, hipEventDisableTiming));
      MGD_HIP(hipEventCreateWithFlags(&bp->ev_out, hipEventDisableTiming));
    }
    MGD_HIP(hipEventRecord(bp->ev_in, user));
    MGD_HIP(hipStreamWaitEvent(bp->aux, bp->ev_in, 0));
    c->stream = bp->aux;
    try {
      block_precond_graph_launch(bp, r, z);
    } catch (...) {
      c->stream = user;
      throw;
    }
    c->stream = user;
    MGD_HIP(hipEventRecord(bp->ev_out, bp->aux));
    MGD_HIP(hipStreamWaitEvent(user, bp->ev_out, 0));
    return;
  }
  block_precond_graph_launch(bp, r, z);
}

void block_precond_graph_launch(block_precond* bp, const double* r, double* z) {
  Ctx* c = bp->ctx;
  auto key = std::make_pair((const void*)r, (void*)z);
  auto it = bp->graphs.find(key);
  if (it == bp->graphs.end()) {
    if (bp->graphs.size() >= 256) {
      for (auto& kv : bp->graphs) hipGraphExecDestroy(kv.second);
      bp->graphs.clear();
    }
    hipGraph_t g = nullptr;
    MGD_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    try {
      block_precond_apply_impl(bp, r, z);
    } catch (...) {
      hipStreamEndCapture(c->stream, &g);
      if (g) hipGraphDestroy(g);
      throw;
    }
    MGD_HIP(hipStreamEndCapture(c->stream, &g));
    hipGraphExec_t ex = nullptr;
    MGD_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    MGD_HIP(hipGraphDestroy(g));
    it = bp->graphs.emplace(key, ex).first;
  }
  MGD_HIP(hipGraphLaunch(it->second, c->stream));
}

bool block_precond_has_first_stage(const block_precond* bp);

// z = M^{-1} r, then y = A z for the system S.  With Schur2 and the shared
// block pattern, the part of A z that does not read z_E runs on a second
// stream beside the last E solve (launches only: usable under capture).
// first_done: w_E* for r was computed by block_precond_first_stage(bp, r).
void block_precond_apply_matvec(block_precond* bp, const double* r, double* z,
                                const BlockSysDev& S, double* y, bool first_done) {
  Ctx* c = bp->ctx;
  MGD_REQUIRE(!first_done || block_precond_has_first_stage(bp),
              "apply: no first stage to skip for this preconditioner");
  // MGD_STEP_OVERLAP=0 keeps the one-kernel matvec after the apply (for comparisons)
  const char* ov = std::getenv("MGD_STEP_OVERLAP");
  const bool split = S.shared && !c->no_alloc && bp->prm.kind == MGD_PC_SCHUR2 &&
                     S.G == bp->G && S.N == bp->N && !(ov && ov[0] == '0');
  if (split) {
    if (!bp->ovl_stream) MGD_HIP(hipStreamCreateWithFlags(&bp->ovl_stream, hipStreamNonBlocking));
    if (!bp->ovl_fork) MGD_HIP(hipEventCreateWithFlags(&bp->ovl_fork, hipEventDisableTiming));
    if (!bp->ovl_join) MGD_HIP(hipEventCreateWithFlags(&bp->ovl_join, hipEventDisableTiming));
  }
  bp->ovl_S = split ? &S : nullptr;
  bp->ovl_y = y;
  bp->ovl_forked = false;
  bp->first_stage = first_done ? 2 : 0;
  try {
    block_precond_apply_impl(bp, r, z);
  } catch (...) {
    bp->ovl_S = nullptr;
    bp->first_stage = 0;
    throw;
  }
  bp->ovl_S = nullptr;
  bp->first_stage = 0;
  if (bp->ovl_forked)
    block_matvec_finish(c, S, z, y);
  else
    block_matvec(c, S, z, nullptr, y);
  bp->ovl_forked = false;
}

// Whether the apply starts with w_E* = A_E^{-1} r_E, a solve that reads r_E
// only (Schur2, its lower form and PCTL, unless every block's coupling to E
// was neglected; inner solves excluded, they decide on the host).
bool block_precond_has_first_stage(const block_precond* bp) {
  const int k = bp->prm.kind;
  if (k != MGD_PC_SCHUR2 && k != MGD_PC_SCHUR2_LOWER && k != MGD_PC_PCTL) return false;
  if (bp->prm.adaptive && k == MGD_PC_SCHUR2 && bp->from_E_weak) return false;
  return bp->prm.inner_tol <= 0;
}

// w_E* = A_E^{-1} r_E for the apply to r that follows with first_done
// (launches only; the buffer it fills is the apply's own, so nothing else
// may apply this preconditioner in between).
void block_precond_first_stage(block_precond* bp, const double* r) {
  MGD_REQUIRE(block_precond_has_first_stage(bp), "apply: no first stage for this preconditioner");
  bp->first_stage = 1;
  try {
    block_precond_apply_impl(bp, r, nullptr);
  } catch (...) {
    bp->first_stage = 0;
    throw;
  }
  bp->first_stage = 0;
}

// Stream and events that order the rest of a Gram-Schmidt update beside the
// first stage of the next apply (created on first use, outside any capture).
void block_precond_side(block_precond* bp, hipStream_t* s, hipEvent_t* fork, hipEvent_t* join) {
  if (!bp->ovl_stream) MGD_HIP(hipStreamCreateWithFlags(&bp->ovl_stream, hipStreamNonBlocking));
  if (!bp->fs_fork) MGD_HIP(hipEventCreateWithFlags(&bp->fs_fork, hipEventDisableTiming));
  if (!bp->fs_join) MGD_HIP(hipEventCreateWithFlags(&bp->fs_join, hipEventDisableTiming));
  *s = bp->ovl_stream;
  *fork = bp->fs_fork;
  *join = bp->fs_join;
}

// Whether a whole GMRES step with this preconditioner may run as one graph:
// graph replay asked for, no host decisions inside the apply, no profiling.
bool block_precond_step_graphable(const block_precond* bp) {
  return bp->prm.use_graph && bp->prm.inner_tol <= 0 && !bp->ctx->profiling &&
         !bp->ctx->no_alloc &&
         bp->prm.kind != MGD_PC_IDENTITY;
}

// Runs `body` (launches only, everything allocated beforehand, the apply in
// its direct form) as one graph, captured on first use for `key`, which must
// hold every pointer and size the launches use.  On the null stream the graph
// runs on a private stream ordered after and before the caller's work.
void block_precond_step_launch(block_precond* bp, const std::vector<uintptr_t>& key,
                               const std::function<void()>& body) {
  Ctx* c = bp->ctx;
  const hipStream_t user = c->stream;
  if (user == nullptr) {
    if (!bp->aux) {
      MGD_HIP(hipStreamCreateWithFlags(&bp->aux, hipStreamNonBlocking));
      MGD_HIP(hipEventCreateWithFlags(&bp->ev_in, hipEventDisableTiming));
      MGD_HIP(hipEventCreateWithFlags(&bp->ev_out, hipEventDisableTiming));
    }
    MGD_HIP(hipEventRecord(bp->ev_in, user));
    MGD_HIP(hipStreamWaitEvent(bp->aux, bp->ev_in, 0));
    c->stream = bp->aux;
  }
  try {
    auto it = bp->step_graphs.find(key);
    if (it == bp->step_graphs.end()) {
      if (bp->step_graphs.size() >= 256) {
        for (auto& kv : bp->step_graphs) hipGraphExecDestroy(kv.second);
        bp->step_graphs.clear();
      }
      hipGraph_t g = nullptr;
      MGD_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
      try {
        body();
      } catch (...) {
        hipStreamEndCapture(c->stream, &g);
        if (g) hipGraphDestroy(g);
        throw;
      }
      MGD_HIP(hipStreamEndCapture(c->stream, &g));
      hipGraphExec_t ex = nullptr;
      MGD_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
      MGD_HIP(hipGraphDestroy(g));
      it = bp->step_graphs.emplace(key, ex).first;
    }
    MGD_HIP(hipGraphLaunch(it->second, c->stream));
  } catch (...) {
    c->stream = user;
    throw;
  }
  if (user == nullptr) {
    c->stream = user;
    MGD_HIP(hipEventRecord(bp->ev_out, bp->aux));
    MGD_HIP(hipStreamWaitEvent(user, bp->ev_out, 0));
  }
}

static void copy_system(block_precond* bp, const mgd_block_system* A) {
  Ctx* c = bp->ctx;
  const int G = A->G, N = A->N;
  const bool tr = bp->prm.transpose != 0;
  bp->blocks.resize(G + 2);
  for (int a = 0; a < G + 2; ++a) {
    if (tr) {
      Csr<double> tmp;
      csr_copy_from(c, &A->blocks[a], tmp);
      transpose(c, tmp, bp->blocks[a]);
    } else {
      csr_copy_from(c, &A->blocks[a], bp->blocks[a]);
    }
    check_structure(c, bp->blocks[a], "copied diagonal block", true);
  }
  bp->d_gE.alloc(c, (size_t)G * N);
  bp->d_Eg.alloc(c, (size_t)G * N);
  bp->d_EI.alloc(c, (size_t)N);
  bp->d_IE.alloc(c, (size_t)N);
  // A^T: D_gE^T sits in the (g, E) position where D_Eg was
  copy_d2d(c, bp->d_gE.get(), tr ? A->d_Eg : A->d_gE, (size_t)G * N);
  copy_d2d(c, bp->d_Eg.get(), tr ? A->d_gE : A->d_Eg, (size_t)G * N);
  copy_d2d(c, bp->d_EI.get(), tr ? A->d_IE : A->d_EI, (size_t)N);
  copy_d2d(c, bp->d_IE.get(), tr ? A->d_EI : A->d_IE, (size_t)N);
  c->sync();
  // Blocks given with one shared pattern keep one in the preconditioner's
  // matvec (copies and sorted transposes of equal patterns are equal).
  bool shared = true;
  for (int a = 1; a < G + 2; ++a)
    shared = shared && A->blocks[a].row_ptr == A->blocks[0].row_ptr &&
             A->blocks[a].col_idx == A->blocks[0].col_idx && A->blocks[a].nnz == A->blocks[0].nnz;
  mgd_block_system view{};
  std::vector<mgd_csr> bl(G + 2);
  for (int a = 0; a < G + 2; ++a) {
    const auto& P = bp->blocks[shared ? 0 : a];
    bl[a] = {bp->blocks[a].n_rows, bp->blocks[a].n_cols, bp->blocks[a].nnz, P.rp.get(), P.ci.get(),
             bp->blocks[a].v.get()};
  }
  view.G = G;
  view.N = N;
  view.blocks = bl.data();
  view.d_gE = bp->d_gE.get();
  view.d_Eg = bp->d_Eg.get();
  view.d_EI = bp->d_EI.get();
  view.d_IE = bp->d_IE.get();
  bp->sys = make_block_sys_dev(&view);
}

// Monolithic CSR of eq. 2.2 (rows [1..G, E, I]), columns sorted.
__global__ void k_mono_len(int G, int N, BlockSysDev S, int* __restrict__ len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= N) return;
  const int nb = S.blk[a].rp[i + 1] - S.blk[a].rp[i];
  const int extra = a < G ? 1 : (a == G ? G + 1 : 1);
  len[(size_t)a * N + i] = nb + extra;
}
__global__ void k_mono_fill(int G, int N, BlockSysDev S, const int* __restrict__ rp,
                            int* __restrict__ ci, double* __restrict__ v, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= N) return;
  int p = rp[(size_t)a * N + i];
  const BlockCsr B = S.blk[a];
  // coupling entries per row: D_gE for a group row, D_Eg (G) and D_EI for E, D_IE for I
  const int extra = a < G ? 1 : (a == G ? G + 1 : 1);
  if (rp[(size_t)a * N + i + 1] - p != (B.rp[i + 1] - B.rp[i]) + extra) {
    atomicOr(err, 1);
    return;
  }
  const int base = a * N;
  if (a == G) {  // D_Eg columns come first (segments 0..G-1)
    for (int g = 0; g < G; ++g) {
      ci[p] = g * N + i;
      v[p++] = S.d_Eg[(size_t)g * N + i];
    }
  }
  if (a == G + 1) {
    ci[p] = G * N + i;
    v[p++] = S.d_IE[i];
  }
  for (int e = B.rp[i]; e < B.rp[i + 1]; ++e) {
    ci[p] = base + B.ci[e];
    v[p++] = B.v[e];
  }
  if (a < G) {
    ci[p] = G * N + i;
    v[p++] = S.d_gE[(size_t)a * N + i];
  }
  if (a == G) {
    ci[p] = (G + 1) * N + i;
    v[p++] = S.d_EI[i];
  }
}

static Csr<double> monolithic(Ctx* c, const BlockSysDev& S) {
  const int G = S.G, N = S.N;
  const long long n = (long long)(G + 2) * N;
  MGD_REQUIRE(n < INT32_MAX, "monolithic matrix too large for int32 indices");
  DBuf<int> len(c, (size_t)n);
  dim3 grid(cdiv(N, 256), G + 2);
  hipLaunchKernelGGL(k_mono_len, grid, dim3(256), 0, c->stream, G, N, S, len.get());
  MGD_CHECK_LAUNCH();
  Csr<double> M;
  M.n_rows = M.n_cols = (int)n;
  M.rp.alloc(c, (size_t)n + 1);
  M.nnz = exclusive_scan_total(c, len.get(), M.rp.get(), (int)n);
  M.ci.alloc(c, (size_t)M.nnz);
  M.v.alloc(c, (size_t)M.nnz);
  hipLaunchKernelGGL(k_mono_fill, grid, dim3(256), 0, c->stream, G, N, S, (const int*)M.rp.get(),
                     M.ci.get(), M.v.get(), c->err_flag());
  MGD_CHECK_LAUNCH();
  c->check_device_errors("monolithic matrix fill");
  return M;
}

// Adaptive strategy (Section 3.5), first level: Definition 1 for every
// coupling block relative to the diagonal of its row block; a coupling is
// neglected when more than sigma_wc N rows are weak, and the neglected ones
// are zeroed in the preconditioner's own copy of the system (so the hats and
// the PCTL residual see the modified matrix).
static void adaptive_couplings(block_precond* bp) {
  Ctx* c = bp->ctx;
  const int G = bp->G, N = bp->N;
  const double th = bp->prm.theta_wc, sig = bp->prm.sigma_wc;
  DBuf<double> dg(c, (size_t)(G + 2) * N);
  for (int a = 0; a < G + 2; ++a) diag_of(c, bp->blocks[a], dg.get() + (size_t)a * N);
  const int nc = 2 * G + 2;
  DBuf<int> cnt(c, (size_t)nc);
  fill<int>(c, cnt.get(), 0, (size_t)nc);
  const dim3 g1(cdiv(N, 256)), b1(256);
  auto count = [&](int slot, const double* d, int row_block) {
    hipLaunchKernelGGL(k_weak_count, g1, b1, 0, c->stream, N, d,
                       (const double*)(dg.get() + (size_t)row_block * N), th, cnt.get() + slot);
    MGD_CHECK_LAUNCH();
  };
  for (int g = 0; g < G; ++g) {
    count(g, bp->d_gE.get() + (size_t)g * N, g);
    count(G + g, bp->d_Eg.get() + (size_t)g * N, G);
  }
  count(2 * G, bp->d_EI.get(), G);
  count(2 * G + 1, bp->d_IE.get(), G + 1);
  std::vector<int> h((size_t)nc);
  copy_d2h(c, h.data(), cnt.get(), (size_t)nc);
  auto weak = [&](int k) { return (double)k > sig * (double)N; };
  bp->cnt_gE.assign(h.begin(), h.begin() + G);
  bp->cnt_Eg.assign(h.begin() + G, h.begin() + 2 * G);
  bp->cnt_EI = h[2 * G];
  bp->cnt_IE = h[2 * G + 1];
  bp->weak_gE.assign(G, 0);
  bp->weak_Eg.assign(G, 0);
  bool all_gE = true, all_Eg = true;
  for (int g = 0; g < G; ++g) {
    bp->weak_gE[g] = weak(bp->cnt_gE[g]);
    bp->weak_Eg[g] = weak(bp->cnt_Eg[g]);
    if (bp->weak_gE[g]) fill<double>(c, bp->d_gE.get() + (size_t)g * N, 0.0, (size_t)N);
    if (bp->weak_Eg[g]) fill<double>(c, bp->d_Eg.get() + (size_t)g * N, 0.0, (size_t)N);
    all_gE = all_gE && bp->weak_gE[g];
    all_Eg = all_Eg && bp->weak_Eg[g];
  }
  bp->weak_EI = weak(bp->cnt_EI);
  bp->weak_IE = weak(bp->cnt_IE);
  if (bp->weak_EI) fill<double>(c, bp->d_EI.get(), 0.0, (size_t)N);
  if (bp->weak_IE) fill<double>(c, bp->d_IE.get(), 0.0, (size_t)N);
  bp->groups_from_E_weak = all_gE;
  bp->into_E_weak_groups = all_Eg;
  bp->from_E_weak = all_gE && bp->weak_IE;
  bp->into_E_weak = all_Eg && bp->weak_EI;
  c->sync();
}

// Second level: Definition 2 on the matrix of every scalar inverse of the
// kind (not PCTL's coarse operator); a matrix with no weakly dominant row is
// inverted by Jacobi iterations (option #1), the others keep V-cycles.
static void adaptive_inverses(block_precond* bp) {
  Ctx* c = bp->ctx;
  const int G = bp->G;
  DBuf<int> cnt(c, (size_t)G + 2);
  fill<int>(c, cnt.get(), 0, (size_t)G + 2);
  for (int r = 0; r < G + 2; ++r) {
    const Csr<double>& A = bp->hier[r]->H.levels[0].A;
    hipLaunchKernelGGL(k_wd_count, dim3(cdiv(A.n_rows, 256)), dim3(256), 0, c->stream, A.n_rows,
                       A.rp.get(), A.ci.get(), A.v.get(), bp->prm.theta_wd, cnt.get() + r);
    MGD_CHECK_LAUNCH();
  }
  std::vector<int> h((size_t)G + 2);
  copy_d2h(c, h.data(), cnt.get(), (size_t)G + 2);
  for (int r = 0; r < G + 2; ++r) {
    bp->wd_count[r] = h[r];
    if (h[r] == 0) {
      const Csr<double>& A = bp->hier[r]->H.levels[0].A;
      bp->jacobi[r] = 1;
      bp->jac_diag[r].alloc(c, (size_t)std::max(A.n_rows, 1));
      diag_of(c, A, bp->jac_diag[r].get());
    }
  }
  c->sync();
}

block_precond* block_precond_create_impl(Ctx* c, const mgd_block_system* A, const block_params* p) {
  auto t0 = std::chrono::steady_clock::now();
  auto bp = std::make_unique<block_precond>();
  bp->ctx = c;
  bp->prm = *p;
  const int G = A->G, N = A->N, kind = p->kind;
  bp->G = G;
  bp->N = N;
  MGD_REQUIRE(kind >= 0 && kind <= MGD_PC_IDENTITY, "unknown preconditioner kind");
  MGD_REQUIRE(p->cycles_rad >= 1 && p->cycles_E >= 1 && p->cycles_I >= 1, "cycles must be >= 1");
  MGD_REQUIRE(p->amg.precision == 0 || p->amg.precision == 1, "precision must be 0 or 1");
  copy_system(bp.get(), A);
  bp->jacobi.assign(G + 3, 0);
  bp->wd_count.assign(G + 3, -1);
  bp->tol_role.assign(G + 3, 0);
  bp->inner_cycles.assign(G + 3, -1);
  if (p->inner_tol > 0)
    for (int r = 0; r < G + 3; ++r)
      bp->tol_role[r] = tolerance_role(kind, r, G, p->option4_steps > 0) ? 1 : 0;
  bp->jac_diag.resize(G + 3);
  if (p->adaptive) {
    MGD_REQUIRE(kind == MGD_PC_PCTL || kind == MGD_PC_SCHUR1 || kind == MGD_PC_SCHUR2,
                "the adaptive strategy applies to PCTL, SCHUR1 and SCHUR2");
    adaptive_couplings(bp.get());
  }
  bp->cycles.assign(G + 3, 1);
  for (int g = 0; g < G; ++g) bp->cycles[g] = p->cycles_rad;
  bp->cycles[G] = p->cycles_E;
  bp->cycles[G + 1] = p->cycles_I;
  bp->cycles[G + 2] = p->cycles_E;
  const Csr<double>* B = bp->blocks.data();
  if (kind == MGD_PC_AMG_MONO) {
    bp->cycles[0] = 1;
    make_hierarchy(bp.get(), 0, monolithic(c, bp->sys));
  } else if (kind != MGD_PC_IDENTITY) {
    DBuf<double> dE(c, N), dI(c, N), dCE(c, N);
    diag_of(c, B[G], dE.get());
    diag_of(c, B[G + 1], dI.get());
    if (kind == MGD_PC_BLOCK_DIAG || kind == MGD_PC_PCTL) {
      for (int a = 0; a < G + 2; ++a) {
        Csr<double> M;
        csr_copy(c, B[a], M);
        make_hierarchy(bp.get(), a, std::move(M));
      }
    } else if (kind == MGD_PC_SCHUR1) {
      Csr<double> CE = hat(c, B[G], bp->d_EI.get(), bp->d_IE.get(), dI.get());
      diag_of(c, CE, dCE.get());
      for (int g = 0; g < G; ++g)
        make_hierarchy(bp.get(), g,
                       hat(c, B[g], bp->d_gE.get() + (size_t)g * N, bp->d_Eg.get() + (size_t)g * N,
                           dCE.get()));
      if (p->option4_steps > 0) {
        Csr<double> AE;  // option #4 iterates with A_E itself (the hat only fixed C^_g)
        csr_copy(c, B[G], AE);
        make_hierarchy(bp.get(), G, std::move(AE));
      } else {
        make_hierarchy(bp.get(), G, std::move(CE));
      }
      Csr<double> AI;
      csr_copy(c, B[G + 1], AI);
      make_hierarchy(bp.get(), G + 1, std::move(AI));
    } else {  // SCHUR2, SCHUR2_LOWER
      for (int g = 0; g < G; ++g)
        make_hierarchy(bp.get(), g,
                       hat(c, B[g], bp->d_gE.get() + (size_t)g * N, bp->d_Eg.get() + (size_t)g * N,
                           dE.get()));
      Csr<double> AE;
      csr_copy(c, B[G], AE);
      make_hierarchy(bp.get(), G, std::move(AE));
      if (p->option4_steps > 0) {
        Csr<double> AI;  // option #4 iterates with A_I itself
        csr_copy(c, B[G + 1], AI);
        make_hierarchy(bp.get(), G + 1, std::move(AI));
      } else {
        make_hierarchy(bp.get(), G + 1, hat(c, B[G + 1], bp->d_IE.get(), bp->d_EI.get(), dE.get()));
      }
    }
    if (kind == MGD_PC_PCTL) {
      // all blocks must share A_E's pattern for eq. 3.1
      DBuf<int> diff(c, 1);
      fill<int>(c, diff.get(), 0, 1);
      for (int a = 0; a < G + 2; ++a) {
        MGD_REQUIRE(B[a].nnz == B[G].nnz, "PCTL needs all diagonal blocks on one pattern");
        hipLaunchKernelGGL(k_pattern_diff, dim3(cdiv(std::max(N + 1, B[G].nnz), 256)), dim3(256), 0,
                           c->stream, N, B[G].nnz, B[G].rp.get(), B[G].ci.get(), B[a].rp.get(),
                           B[a].ci.get(), diff.get());
        MGD_CHECK_LAUNCH();
      }
      MGD_REQUIRE(read1(c, diff.get()) == 0, "PCTL needs all diagonal blocks on one pattern");
      bp->p.alloc(c, (size_t)(G + 1) * N);
      DBuf<double> rhs(c, N);
      bp->p_cycles.clear();
      for (int g = 0; g <= G; ++g) {
        const int role = g < G ? g : G + 1;
        const double* dcol = g < G ? bp->d_gE.get() + (size_t)g * N : bp->d_IE.get();
        hipLaunchKernelGGL(k_neg, dim3(cdiv(N, 256)), dim3(256), 0, c->stream, N, dcol, rhs.get());
        MGD_CHECK_LAUNCH();
        bp->p_cycles.push_back(solve_to_tol(bp.get(), bp->hier[role].get(), rhs.get(),
                                            bp->p.get() + (size_t)g * N, p->pctl_p_tol,
                                            p->pctl_p_maxcycles));
      }
      Csr<double> Ac;
      csr_copy(c, B[G], Ac);
      hipLaunchKernelGGL(k_pctl_coarse, dim3(cdiv(N, 256)), dim3(256), 0, c->stream, G, N, bp->sys,
                         (const double*)bp->p.get(), Ac.v.get());
      MGD_CHECK_LAUNCH();
      make_hierarchy(bp.get(), G + 2, std::move(Ac));
      // the FP64 unions used for the p solves are not needed by an FP32 apply
      if (p->amg.precision == 1)
        for (auto& h : bp->hier)
          if (h) h->u64.reset();
    }
  }
  if (p->adaptive) adaptive_inverses(bp.get());
  if (p->amg.precision == 1 && kind != MGD_PC_IDENTITY)
    build_exec<float>(bp.get(), bp->x32);
  else
    build_exec<double>(bp.get(), bp->x64);
  c->sync();
  bp->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return bp.release();
}
