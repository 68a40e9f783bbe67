// Vector primitives: scans, fills, casts and deterministic reductions.
//
// Reductions split the index range over a FIXED number of workgroups with a
// grid-stride loop, reduce each workgroup with wavefront shuffles and LDS,
// and sum the per-workgroup partials in index order in a second kernel, so
// the result depends only on n, never on scheduling.
#include "kernels.hpp"

namespace mgd {

// ---------------------------------------------------------------------------
// wavefront / workgroup reductions (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a 256-thread workgroup; result valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* lds /*[4]*/) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// scan
// ---------------------------------------------------------------------------
constexpr int kScanTile = 2048;  // 256 threads x 8 items

__global__ void __launch_bounds__(256) k_tile_sums(const int* __restrict__ in, int n,
                                                   int* __restrict__ sums) {
  __shared__ int lds[4];
  const long base = (long)blockIdx.x * kScanTile;
  int s = 0;
  for (int k = threadIdx.x; k < kScanTile; k += 256) {
    long i = base + k;
    if (i < n) s += in[i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

// Exclusive scan of one tile with an additive base; writes out[i] for
// i < n and, from the block holding the last element, out[n] = total.
__global__ void __launch_bounds__(256) k_tile_scan(const int* __restrict__ in, int n,
                                                   const int* __restrict__ base_of_tile,
                                                   int* __restrict__ out) {
  __shared__ int lds[256];
  const long base = (long)blockIdx.x * kScanTile;
  const int t = threadIdx.x;
  int v[8];
  int s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    long i = base + t * 8 + k;
    v[k] = (i < n) ? in[i] : 0;
    s += v[k];
  }
  lds[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over 256 thread sums
  for (int off = 1; off < 256; off <<= 1) {
    int add = (t >= off) ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  int run = (t ? lds[t - 1] : 0) + (base_of_tile ? base_of_tile[blockIdx.x] : 0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    long i = base + t * 8 + k;
    if (i < n) out[i] = run;
    run += v[k];
    if (i == n - 1) out[n] = run;
  }
}

__global__ void k_set_zero_total(int* out) { out[0] = 0; }

void exclusive_scan(Ctx* c, const int* in, int* out, int n) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_set_zero_total, dim3(1), dim3(1), 0, c->stream, out);
    MGD_CHECK_LAUNCH();
    return;
  }
  const int tiles = cdiv(n, kScanTile);
  if (tiles == 1) {
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(256), 0, c->stream, in, n, nullptr, out);
    MGD_CHECK_LAUNCH();
    return;
  }
  DBuf<int> sums(c, tiles), sums_scan(c, (size_t)tiles + 1);
  hipLaunchKernelGGL(k_tile_sums, dim3(tiles), dim3(256), 0, c->stream, in, n, sums.get());
  MGD_CHECK_LAUNCH();
  exclusive_scan(c, sums.get(), sums_scan.get(), tiles);
  hipLaunchKernelGGL(k_tile_scan, dim3(tiles), dim3(256), 0, c->stream, in, n,
                     (const int*)sums_scan.get(), out);
  MGD_CHECK_LAUNCH();
  // temporaries are released only after the stream has consumed them
  c->sync();
}

int exclusive_scan_total(Ctx* c, const int* in, int* out, int n) {
  exclusive_scan(c, in, out, n);
  return read1(c, out + (n > 0 ? n : 0));
}

// ---------------------------------------------------------------------------
// device copy
// ---------------------------------------------------------------------------
__global__ void k_copy_words(uint32_t* __restrict__ d, const uint32_t* __restrict__ s, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}
__global__ void k_copy_bytes(uint8_t* __restrict__ d, const uint8_t* __restrict__ s, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}
void device_copy(Ctx* c, void* dst, const void* src, size_t bytes) {
  if (!bytes) return;
  const bool words = bytes % 4 == 0 && ((uintptr_t)dst % 4) == 0 && ((uintptr_t)src % 4) == 0;
  const size_t n = words ? bytes / 4 : bytes;
  const int g = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192);
  if (words)
    hipLaunchKernelGGL(k_copy_words, dim3(g), dim3(kBlock), 0, c->stream, (uint32_t*)dst,
                       (const uint32_t*)src, n);
  else
    hipLaunchKernelGGL(k_copy_bytes, dim3(g), dim3(kBlock), 0, c->stream, (uint8_t*)dst,
                       (const uint8_t*)src, n);
  MGD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// fill / cast
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* __restrict__ p, T v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}
template <typename T>
void fill(Ctx* c, T* p, T v, size_t n) {
  if (!n) return;
  int g = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 65535 * 4);
  hipLaunchKernelGGL(k_fill<T>, dim3(g), dim3(kBlock), 0, c->stream, p, v, n);
  MGD_CHECK_LAUNCH();
}
template void fill<int>(Ctx*, int*, int, size_t);
template void fill<unsigned>(Ctx*, unsigned*, unsigned, size_t);
template void fill<int8_t>(Ctx*, int8_t*, int8_t, size_t);
template void fill<uint8_t>(Ctx*, uint8_t*, uint8_t, size_t);
template void fill<double>(Ctx*, double*, double, size_t);
template void fill<float>(Ctx*, float*, float, size_t);

template <typename D, typename S>
__global__ void k_cast(D* __restrict__ d, const S* __restrict__ s, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = (D)s[i];
}
template <typename D, typename S>
void cast_copy(Ctx* c, D* dst, const S* src, size_t n, int cls) {
  if (!n) return;
  ProfScope ps(c, cls, (double)n * (sizeof(D) + sizeof(S)));
  int g = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 65535 * 4);
  hipLaunchKernelGGL((k_cast<D, S>), dim3(g), dim3(kBlock), 0, c->stream, dst, src, n);
  MGD_CHECK_LAUNCH();
}
template void cast_copy<float, double>(Ctx*, float*, const double*, size_t, int);
template void cast_copy<double, float>(Ctx*, double*, const float*, size_t, int);
template void cast_copy<double, double>(Ctx*, double*, const double*, size_t, int);
template void cast_copy<float, float>(Ctx*, float*, const float*, size_t, int);

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
static int red_grid(size_t n) {
  size_t g = (n + kBlock - 1) / kBlock;
  return (int)std::max<size_t>(1, std::min<size_t>(g, kRedBlocks));
}

// Index of element i's slot in the t-th grid stride counted from the END of the
// vector: a sweep that follows a forward sweep over the same vectors starts on
// the data that sweep read last, which the device's last-level cache (256 MB)
// still holds.
__device__ __forceinline__ size_t rev_stride_index(size_t t, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256;
  const size_t last = (n - 1) / stride;
  return (last - t) * stride + blockIdx.x * (size_t)256 + threadIdx.x;
}

// Final stage: out[j] = sum_b partial[j*nb + b] for b ascending over a fixed
// tree: thread t sums b = t, t+256, ...; then the workgroup tree.
__global__ void __launch_bounds__(256) k_red_final(const double* __restrict__ partial, int nb,
                                                   double* __restrict__ out) {
  __shared__ double lds[4];
  const double* p = partial + (size_t)blockIdx.x * nb;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += p[b];
  s = block_sum256(s, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_dot(const double* __restrict__ x,
                                             const double* __restrict__ y, size_t n,
                                             double* __restrict__ partial) {
  __shared__ double lds[4];
  double s = 0.0;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    s += x[i] * y[i];
  s = block_sum256(s, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void dot_dev(Ctx* c, RedWork& w, const double* x, const double* y, size_t n, double* out) {
  w.ensure(c);
  ProfScope ps(c, KC_ORTH, 16.0 * n);
  int g = red_grid(n);
  hipLaunchKernelGGL(k_dot, dim3(g), dim3(256), 0, c->stream, x, y, n, w.partial.get());
  MGD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_red_final, dim3(1), dim3(256), 0, c->stream, (const double*)w.partial.get(),
                     g, out);
  MGD_CHECK_LAUNCH();
}

constexpr int kMaxJ = 32;

// Arnoldi orthogonalisation passes (classical Gram-Schmidt with selective
// reorthogonalisation, Daniel-Gragg-Kaufman-Stewart criterion eta = 1/sqrt 2):
// mode 0: h[j] = V_j . w,                            h[J] = w . w
// mode 1: w -= sum h_in[j] V_j;  h[j] = V_j . w_new, h[J] = w_new . w_new
// (the third pass, k_orth_finish, applies the second projection when needed
// and normalises in the same sweep)
template <int MODE, int JB>
__global__ void __launch_bounds__(256) k_mdot(const double* __restrict__ V, size_t ldv, int J,
                                              const double* __restrict__ h_in,
                                              const double* __restrict__ h_first,
                                              double* __restrict__ w, size_t n,
                                              double* __restrict__ partial, int nb) {
  __shared__ double lds[4];
  (void)h_first;
  double acc[JB + 1];
  double hv[JB];
#pragma unroll
  for (int j = 0; j < JB; ++j) {
    acc[j] = 0.0;
    hv[j] = (MODE != 0 && j < J) ? h_in[j] : 0.0;
  }
  acc[JB] = 0.0;
  double nacc = 0.0;
  // mode 0 sweeps forward, mode 1 (which follows it) backward
  const size_t nt = n ? (n - 1) / ((size_t)gridDim.x * 256) + 1 : 0;
  for (size_t t = 0; t < nt; ++t) {
    const size_t i = MODE == 0 ? t * (size_t)gridDim.x * 256 + blockIdx.x * (size_t)256 + threadIdx.x
                               : rev_stride_index(t, n);
    if (i >= n) continue;
    double wi = w[i];
    // all loads of the basis column first, so they are in flight together
    double vj[JB];
#pragma unroll
    for (int j = 0; j < JB; ++j)
      if (j < J) vj[j] = V[j * ldv + i];
    if (MODE == 0) {
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < J) acc[j] += vj[j] * wi;
      nacc += wi * wi;
    } else {
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < J) wi -= hv[j] * vj[j];
      w[i] = wi;
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < J) acc[j] += vj[j] * wi;
      nacc += wi * wi;
    }
  }
#pragma unroll
  for (int j = 0; j < JB; ++j) {
    if (j < J) {  // J is uniform: every thread takes the same branches around the barriers
      double s = block_sum256(acc[j], lds);
      if (threadIdx.x == 0) partial[(size_t)j * nb + blockIdx.x] = s;
    }
  }
  double s = block_sum256(nacc, lds);
  if (threadIdx.x == 0) partial[(size_t)J * nb + blockIdx.x] = s;
}

struct MdotArgs {
  const double* V;
  size_t ldv;
  int J;
  const double* h_in;
  const double* h_first;
  double* w;
  size_t n;
  double* partial;
  int nb;
};
// register arrays sized to the next power of two >= J keep occupancy up for short bases
static int mdot_jb(int J) { return J <= 4 ? 4 : J <= 8 ? 8 : J <= 16 ? 16 : 32; }
template <int MODE>
static void launch_mdot(Ctx* c, const MdotArgs& a) {
  const dim3 g(a.nb), b(256);
#define MGD_MDOT(JB)                                                                             \
  hipLaunchKernelGGL((k_mdot<MODE, JB>), g, b, 0, c->stream, a.V, a.ldv, a.J, a.h_in, a.h_first, \
                     a.w, a.n, a.partial, a.nb)
  if (a.J <= 4)
    MGD_MDOT(4);
  else if (a.J <= 8)
    MGD_MDOT(8);
  else if (a.J <= 16)
    MGD_MDOT(16);
  else
    MGD_MDOT(32);
#undef MGD_MDOT
  MGD_CHECK_LAUNCH();
}

void mdot_dev(Ctx* c, RedWork& w, const double* V, size_t ldv, int J, const double* wv, size_t n,
              double* h) {
  MGD_REQUIRE(J >= 1 && J < kMaxJ, "mdot: J out of range");
  w.ensure(c);
  ProfScope ps(c, KC_ORTH, 8.0 * n * (J + 1), ksym(c, "k_mdot", {"0", std::to_string(mdot_jb(J))}));
  int g = red_grid(n);
  MdotArgs a{V, ldv, J, nullptr, nullptr, const_cast<double*>(wv), n, w.partial.get(), g};
  launch_mdot<0>(c, a);
  MGD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_red_final, dim3(J + 1), dim3(256), 0, c->stream,
                     (const double*)w.partial.get(), g, h);
  MGD_CHECK_LAUNCH();
}

void update_mdot_dev(Ctx* c, RedWork& w, const double* V, size_t ldv, int J, const double* h,
                     double* wv, size_t n, double* h2) {
  MGD_REQUIRE(J >= 1 && J < kMaxJ, "mdot: J out of range");
  w.ensure(c);
  ProfScope ps(c, KC_ORTH, 8.0 * n * (J + 2), ksym(c, "k_mdot", {"1", std::to_string(mdot_jb(J))}));
  int g = red_grid(n);
  MdotArgs a{V, ldv, J, h, nullptr, wv, n, w.partial.get(), g};
  launch_mdot<1>(c, a);
  MGD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_red_final, dim3(J + 1), dim3(256), 0, c->stream,
                     (const double*)w.partial.get(), g, h2);
  MGD_CHECK_LAUNCH();
}

// Third pass of one Arnoldi step.  k_arnoldi_col forms the Hessenberg column
// from the two projections: reorthogonalise when h2[J] < h1[J] / 2 (the first
// projection removed more than half of the squared norm); then the column is
// h1 + h2, and the new norm comes from Pythagoras, ||w''||^2 = ||w'||^2 -
// sum h2[j]^2 (the second projection's coefficients are tiny, so this loses
// nothing), else the column is h1 with norm ||w'||.  hcol[J] is the scale used
// (1 when the difference is not positive), hcol[J+1] = 1 when reorthogonalised.
__global__ void k_arnoldi_col(const double* __restrict__ h1, const double* __restrict__ h2, int J,
                              double* __restrict__ hcol) {
  const bool re = h2[J] < 0.5 * h1[J];
  const int j = threadIdx.x;
  if (j < J) hcol[j] = re ? h1[j] + h2[j] : h1[j];
  if (j == 0) {
    double est = h2[J];
    if (re)
      for (int k = 0; k < J; ++k) est = est - h2[k] * h2[k];
    hcol[J] = est > 0.0 ? sqrt(est) : 1.0;
    hcol[J + 1] = re ? 1.0 : 0.0;
  }
}
// v = (w' - [reorthogonalised] sum h2[j] V_j) / hcol[J] in place, and the
// exact ||w''||^2 of the unscaled vector per block (the host compares it with
// the scale and corrects the rare mismatch)
template <int JB>
__global__ void __launch_bounds__(256) k_orth_finish(const double* __restrict__ V, size_t ldv,
                                                     int J, const double* __restrict__ h2,
                                                     const double* __restrict__ hcol,
                                                     double* __restrict__ w, size_t n,
                                                     double* __restrict__ partial) {
  __shared__ double lds[4];
  const bool re = hcol[J + 1] != 0.0;  // uniform
  const double nr = hcol[J];
  double hv[JB];
#pragma unroll
  for (int j = 0; j < JB; ++j) hv[j] = (re && j < J) ? h2[j] : 0.0;
  double nacc = 0.0;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    double wi = w[i];
    if (re) {
      double vj[JB];
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < J) vj[j] = V[j * ldv + i];
#pragma unroll
      for (int j = 0; j < JB; ++j)
        if (j < J) wi -= hv[j] * vj[j];
    }
    nacc += wi * wi;
    w[i] = wi / nr;
  }
  double s = block_sum256(nacc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void orth_finish_dev(Ctx* c, RedWork& w, const double* V, size_t ldv, int J, const double* h1,
                     const double* h2, double* hcol, double* wv, size_t n) {
  MGD_REQUIRE(J >= 1 && J < kMaxJ, "mdot: J out of range");
  w.ensure(c);
  hipLaunchKernelGGL(k_arnoldi_col, dim3(1), dim3(64), 0, c->stream, h1, h2, J, hcol);
  MGD_CHECK_LAUNCH();
  // algorithmic bytes of the reorthogonalised case (the usual one)
  ProfScope ps(c, KC_ORTH, 8.0 * n * (J + 2), ksym(c, "k_orth_finish", {std::to_string(mdot_jb(J))}));
  const int g = red_grid(n);
#define MGD_ORTH(JB)                                                                      \
  hipLaunchKernelGGL((k_orth_finish<JB>), dim3(g), dim3(256), 0, c->stream, V, ldv, J, h2, \
                     (const double*)hcol, wv, n, w.partial.get())
  if (J <= 4)
    MGD_ORTH(4);
  else if (J <= 8)
    MGD_ORTH(8);
  else if (J <= 16)
    MGD_ORTH(16);
  else
    MGD_ORTH(32);
#undef MGD_ORTH
  MGD_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_red_final, dim3(1), dim3(256), 0, c->stream, (const double*)w.partial.get(),
                     g, hcol + J + 2);
  MGD_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Delayed reorthogonalisation (two sweeps per Arnoldi step)
// ---------------------------------------------------------------------------
// Sweep 1: per block partial sums of a_k = V_k . vj, b_k = V_k . w (k < F),
// b_F = vj . w, ww = w . w, vv = vj . vj; outputs [0, F) a, [F, 2F) b, 2F b_F,
// 2F+1 ww, 2F+2 vv (the vj terms are zero without vj).
template <int JB, bool PROV>
__global__ void __launch_bounds__(256) k_dcgs_dots(const double* __restrict__ V, size_t ldv, int F,
                                                   const double* __restrict__ vj,
                                                   const double* __restrict__ w, size_t n,
                                                   double* __restrict__ partial, int nb) {
  __shared__ double lds[4];
  double aa[JB], bb[JB];
#pragma unroll
  for (int k = 0; k < JB; ++k) aa[k] = bb[k] = 0.0;
  double bF = 0.0, ww = 0.0, vv = 0.0;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double wi = w[i];
    const double vi = PROV ? vj[i] : 0.0;
    double vk[JB];
#pragma unroll
    for (int k = 0; k < JB; ++k)
      if (k < F) vk[k] = V[k * ldv + i];
#pragma unroll
    for (int k = 0; k < JB; ++k) {
      if (k < F) {
        if (PROV) aa[k] += vk[k] * vi;
        bb[k] += vk[k] * wi;
      }
    }
    if (PROV) {
      bF += vi * wi;
      vv += vi * vi;
    }
    ww += wi * wi;
  }
#pragma unroll
  for (int k = 0; k < JB; ++k) {
    if (k < F) {  // F is uniform: every thread takes the same branches around the barriers
      const double sa = PROV ? block_sum256(aa[k], lds) : 0.0;
      const double sb = block_sum256(bb[k], lds);
      if (threadIdx.x == 0) {
        partial[(size_t)k * nb + blockIdx.x] = sa;
        partial[(size_t)(F + k) * nb + blockIdx.x] = sb;
      }
    }
  }
  const double s1 = PROV ? block_sum256(bF, lds) : 0.0;
  const double s2 = block_sum256(ww, lds);
  const double s3 = PROV ? block_sum256(vv, lds) : 0.0;
  if (threadIdx.x == 0) {
    partial[(size_t)(2 * F) * nb + blockIdx.x] = s1;
    partial[(size_t)(2 * F + 1) * nb + blockIdx.x] = s2;
    partial[(size_t)(2 * F + 2) * nb + blockIdx.x] = s3;
  }
}

// The step's coefficients from the dots (one thread).
__global__ void k_dcgs_coef(int F, int prov, const double* __restrict__ d,
                            double* __restrict__ coef) {
  if (threadIdx.x != 0) return;
  const double* a = d;
  const double* b = d + F;
  double beta = 1.0;
  for (int k = 0; k < 64; ++k) coef[k] = 0.0;
  if (prov) {
    double s = 0.0;
    for (int k = 0; k < F; ++k) s = s + a[k] * a[k];
    const double b2 = d[2 * F + 2] - s;
    beta = b2 > 0.0 ? sqrt(b2) : 1.0;
    for (int k = 0; k < F; ++k) coef[k] = a[k];
  }
  double hs = 0.0;
  for (int k = 0; k < F; ++k) {
    coef[32 + k] = b[k];
    hs = hs + b[k] * b[k];
  }
  if (prov) {
    double t = d[2 * F];
    for (int k = 0; k < F; ++k) t = t - a[k] * b[k];
    const double hF = t / beta;
    coef[32 + F] = hF;
    hs = hs + hF * hF;
  }
  const double al2 = d[2 * F + 1] - hs;
  coef[64] = beta;
  coef[65] = al2 > 0.0 ? sqrt(al2) : 1.0;
}

// Sweep 2: vj <- (vj - sum a_k V_k) / beta; w <- (w - sum h_k V_k - h_F vj_new) / alpha,
// with per block partial sums of |vj_new|^2 and |w before the division|^2
// (written at partial[poff + block] and partial[nb + poff + block]).  The
// sweep covers m entries: the k-th is entry base + k, plus gap from k = lo on
// (a range with one hole).
template <int JB, bool PROV>
__global__ void __launch_bounds__(256) k_dcgs_update(const double* __restrict__ V, size_t ldv,
                                                     int F, const double* __restrict__ coef,
                                                     double* __restrict__ vj,
                                                     double* __restrict__ w, size_t m,
                                                     size_t base, size_t lo, size_t gap,
                                                     double* __restrict__ partial, int nb,
                                                     int poff) {
  __shared__ double lds[4];
  double ca[JB], ch[JB];
#pragma unroll
  for (int k = 0; k < JB; ++k) {
    ca[k] = (PROV && k < F) ? coef[k] : 0.0;
    ch[k] = k < F ? coef[32 + k] : 0.0;
  }
  const double hF = PROV ? coef[32 + F] : 0.0;
  const double beta = coef[64], alpha = coef[65];
  double sv = 0.0, sw = 0.0;
  // backward: the dots sweep before it ran forward over the same vectors
  const size_t nt = m ? (m - 1) / ((size_t)gridDim.x * 256) + 1 : 0;
  for (size_t t = 0; t < nt; ++t) {
    const size_t k = rev_stride_index(t, m);
    if (k >= m) continue;
    const size_t i = base + k + (k >= lo ? gap : 0);
    double vk[JB];
#pragma unroll
    for (int k = 0; k < JB; ++k)
      if (k < F) vk[k] = V[k * ldv + i];
    double wi = w[i];
    double vn = 0.0;
    if (PROV) {
      double vi = vj[i];
#pragma unroll
      for (int k = 0; k < JB; ++k)
        if (k < F) vi -= ca[k] * vk[k];
      vn = vi / beta;
      vj[i] = vn;
      sv += vn * vn;
    }
#pragma unroll
    for (int k = 0; k < JB; ++k)
      if (k < F) wi -= ch[k] * vk[k];
    if (PROV) wi -= hF * vn;
    sw += wi * wi;
    w[i] = wi / alpha;
  }
  const double s1 = PROV ? block_sum256(sv, lds) : 0.0;
  const double s2 = block_sum256(sw, lds);
  if (threadIdx.x == 0) {
    partial[(size_t)poff + blockIdx.x] = s1;
    partial[(size_t)nb + poff + blockIdx.x] = s2;
  }
}

void dcgs_step_dev(Ctx* c, RedWork& w, const double* V, size_t ldv, int F, double* vj,
                   double* wv, size_t n, double* dots, double* coef, const DcgsSplit* split) {
  MGD_REQUIRE(F >= 1 && F <= 31, "dcgs: F out of range");
  w.ensure(c);
  const bool prov = vj != nullptr;
  const int jb = mdot_jb(F);
  // with 32-vector register arrays two workgroups fit a compute unit: one
  // round of resident workgroups
  const int g = jb == 32 ? std::min(red_grid(n), kRedBlocks / 2) : red_grid(n);
  {
    ProfScope ps(c, KC_ORTH, 8.0 * n * (F + (prov ? 2 : 1)),
                 ksym(c, "k_dcgs_dots", {std::to_string(jb), prov ? "true" : "false"}));
#define MGD_DOTS(JB, P)                                                                         \
  hipLaunchKernelGGL((k_dcgs_dots<JB, P>), dim3(g), dim3(256), 0, c->stream, V, ldv, F,           \
                     (const double*)vj, (const double*)wv, n, w.partial.get(), g)
#define MGD_DOTS_P(JB) \
  if (prov)            \
    MGD_DOTS(JB, true);  \
  else                 \
    MGD_DOTS(JB, false)
    if (jb == 4) {
      MGD_DOTS_P(4);
    } else if (jb == 8) {
      MGD_DOTS_P(8);
    } else if (jb == 16) {
      MGD_DOTS_P(16);
    } else {
      MGD_DOTS_P(32);
    }
#undef MGD_DOTS_P
#undef MGD_DOTS
    MGD_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_red_final, dim3(2 * F + 3), dim3(256), 0, c->stream,
                     (const double*)w.partial.get(), g, dots);
  hipLaunchKernelGGL(k_dcgs_coef, dim3(1), dim3(64), 0, c->stream, F, prov ? 1 : 0,
                     (const double*)dots, coef);
  MGD_CHECK_LAUNCH();
  // one update sweep over m entries (see k_dcgs_update), partials at poff
  auto update = [&](size_t m, size_t base, size_t lo, size_t gap, int gu, int nb, int poff,
                    hipStream_t s) {
    ProfScope ps(c, KC_ORTH, 8.0 * m * (F + (prov ? 4 : 2)),
                 ksym(c, "k_dcgs_update", {std::to_string(jb), prov ? "true" : "false"}), -1, s);
#define MGD_UPD(JB, P)                                                                        \
  hipLaunchKernelGGL((k_dcgs_update<JB, P>), dim3(gu), dim3(256), 0, s, V, ldv, F,              \
                     (const double*)coef, vj, wv, m, base, lo, gap, w.partial.get(), nb, poff)
#define MGD_UPD_P(JB) \
  if (prov)           \
    MGD_UPD(JB, true);  \
  else                \
    MGD_UPD(JB, false)
    if (jb == 4) {
      MGD_UPD_P(4);
    } else if (jb == 8) {
      MGD_UPD_P(8);
    } else if (jb == 16) {
      MGD_UPD_P(16);
    } else {
      MGD_UPD_P(32);
    }
#undef MGD_UPD_P
#undef MGD_UPD
    MGD_CHECK_LAUNCH();
  };
  int nb = g;
  if (!split) {
    update(n, 0, n, 0, g, g, 0, c->stream);
  } else {
    MGD_REQUIRE(split->lo < split->hi && split->hi <= n && split->side && split->fork &&
                    split->join,
                "dcgs: bad split");
    const size_t mh = split->hi - split->lo, mr = n - mh;
    const int gh = red_grid(mh), gr = mr ? red_grid(mr) : 0;
    nb = gh + gr;
    MGD_REQUIRE(2 * (size_t)nb <= (size_t)kRedBlocks * 66, "dcgs: too many partials");
    update(mh, split->lo, mh, 0, gh, nb, 0, c->stream);
    MGD_HIP(hipEventRecord(split->fork, c->stream));
    MGD_HIP(hipStreamWaitEvent(split->side, split->fork, 0));
    if (mr) update(mr, 0, split->lo, mh, gr, nb, gh, split->side);
    MGD_HIP(hipEventRecord(split->join, split->side));
    if (split->beside) split->beside();
    MGD_HIP(hipStreamWaitEvent(c->stream, split->join, 0));
  }
  hipLaunchKernelGGL(k_red_final, dim3(2), dim3(256), 0, c->stream, (const double*)w.partial.get(),
                     nb, coef + 66);
  MGD_CHECK_LAUNCH();
}

__global__ void k_scale_vec(double a, double* __restrict__ v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    v[i] = v[i] * a;
}
void scale_dev(Ctx* c, double a, double* v, size_t n) {
  ProfScope ps(c, KC_ORTH, 16.0 * n, ksym(c, "k_scale_vec", {}));
  int g = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_scale_vec, dim3(g), dim3(kBlock), 0, c->stream, a, v, n);
  MGD_CHECK_LAUNCH();
}

__global__ void k_combine(const double* __restrict__ Z, size_t ldz, int K,
                          const double* __restrict__ y, double* __restrict__ x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double s = x[i];
    for (int k = 0; k < K; ++k) s += y[k] * Z[k * ldz + i];
    x[i] = s;
  }
}
void combine_dev(Ctx* c, const double* Z, size_t ldz, int K, const double* y, double* x,
                 size_t n) {
  if (K <= 0) return;
  ProfScope ps(c, KC_ORTH, 8.0 * n * (K + 2));
  int g = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_combine, dim3(g), dim3(kBlock), 0, c->stream, Z, ldz, K, y, x, n);
  MGD_CHECK_LAUNCH();
}

__global__ void k_rsub(const double* __restrict__ b, double* __restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] = b[i] - y[i];
}
void rsub(Ctx* c, const double* b, double* y, size_t n) {
  ProfScope ps(c, KC_VEC, 24.0 * n);
  int g = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_rsub, dim3(g), dim3(kBlock), 0, c->stream, b, y, n);
  MGD_CHECK_LAUNCH();
}

__global__ void k_scale_copy(double* __restrict__ y, const double* __restrict__ x, double a,
                             size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}
void scale_copy(Ctx* c, double* y, const double* x, double a, size_t n) {
  ProfScope ps(c, KC_VEC, 16.0 * n);
  int g = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_scale_copy, dim3(g), dim3(kBlock), 0, c->stream, y, x, a, n);
  MGD_CHECK_LAUNCH();
}
__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}
void axpy(Ctx* c, double* y, const double* x, double a, size_t n) {
  ProfScope ps(c, KC_VEC, 24.0 * n);
  int g = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_axpy, dim3(g), dim3(kBlock), 0, c->stream, y, x, a, n);
  MGD_CHECK_LAUNCH();
}

}  // namespace mgd
