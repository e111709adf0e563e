// HIP kernels of libffx for gfx950 (CDNA4, 64-wide wavefronts).
//
// The state is the dim_a x dim_b matrix Gamma (alpha-major) of interleaved
// complex numbers (re, im): complex128 or complex64.
//
// Givens sweeps (Sec. 3.2.3).  A window pass applies a list of adjacent Givens
// rotations whose orbitals all lie in one window [a, a+W) of one spin.  Such
// rotations only mix configurations that agree outside the window, so each
// class of those configurations (C(W, m) members, m = electrons in the window)
// is loaded once into registers, every rotation of the pass is applied in
// registers, and the class is stored once: one HBM round trip for the whole
// list.  The member pairs touched by a rotation on (p, p+1) are compile-time
// constants for given (W, m, p), so the register arrays are indexed
// statically.
//   alpha pass: a block owns one alpha class and 256 consecutive columns;
//               lanes run along the contiguous beta index (coalesced).
//   beta pass:  a wave owns 64 beta classes of one row that share m; lanes of
//               classes with consecutive low patterns touch consecutive columns.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <utility>

#include "dev_common.h"
#include "device.h"

namespace ffx {
namespace dev {

// ---------------------------------------------------------------------------
// window passes
// ---------------------------------------------------------------------------
// Row bases are wave-uniform (scalar registers) and the lane part is one
// 32-bit byte offset shared by every member, so each access is a scalar-base +
// vector-offset load with no per-member 64-bit address registers.
template <class V>
__device__ __forceinline__ const V& at_off(const V* base, uint32_t off) {
  return *(const V*)((const char*)base + off);
}
template <class V>
__device__ __forceinline__ V& at_off(V* base, uint32_t off) {
  return *(V*)((char*)base + off);
}
template <class V, class R, int... K>
__device__ __forceinline__ void load_alpha(V* v, const V* __restrict__ vec, int64_t dim_b, const int* __restrict__ t,
                                           uint32_t off, std::integer_sequence<int, K...>) {
  ((v[K] = at_off(vec + (int64_t)t[K * 64] * dim_b, off)), ...);
}
template <class V, class R, int... K>
__device__ __forceinline__ void store_alpha(const V* v, V* __restrict__ vec, int64_t dim_b, const int* t,
                                            uint32_t off, const V* __restrict__ phase,
                                            std::integer_sequence<int, K...>) {
  if (phase)
    ((at_off(vec + (int64_t)t[K * 64] * dim_b, off) = cmul<V, R>(v[K], phase[t[K * 64]])), ...);
  else
    ((at_off(vec + (int64_t)t[K * 64] * dim_b, off) = v[K]), ...);
}
template <class V, class R, int... K>
__device__ __forceinline__ void load_beta(V* v, const V* __restrict__ rowp, const int* __restrict__ t,
                                          std::integer_sequence<int, K...>) {
  ((v[K] = rowp[t[K * 64]]), ...);
}
// The member columns are re-read from the (cache-resident) table at store time
// instead of being kept live across the rotations: at W = 8 they would cost 70
// extra registers per lane.
template <class V, class R, int... K>
__device__ __forceinline__ void store_beta(const V* v, V* __restrict__ rowp, const int* t,
                                           const V* __restrict__ phase, std::integer_sequence<int, K...>) {
  const volatile int* tv = t;
  if (phase)
    ((rowp[tv[K * 64]] = cmul<V, R>(v[K], phase[tv[K * 64]])), ...);
  else
    ((rowp[tv[K * 64]] = v[K]), ...);
}

template <int W, int M, bool REAL, class R>
__device__ __forceinline__ void alpha_body(typename V2T<R>::type* __restrict__ vec, int64_t dim_b,
                                           const int* __restrict__ t, uint32_t col,
                                           const RotDev* __restrict__ rots, int nrot,
                                           const typename V2T<R>::type* __restrict__ phase) {
  using V = typename V2T<R>::type;
  constexpr int C = cbinom(W, M);
  V v[C];
  const uint32_t off = col * (uint32_t)sizeof(V);
  load_alpha<V, R>(v, vec, dim_b, t, off, std::make_integer_sequence<int, C>{});
  apply_rots<W, M, REAL, typename V2T<R>::type>(v, rots, nrot);
  store_alpha<V, R>(v, vec, dim_b, t, off, phase, std::make_integer_sequence<int, C>{});
}

template <int W, int M, bool REAL, class R>
__device__ __forceinline__ void beta_body(typename V2T<R>::type* __restrict__ rowp,
                                          const int* __restrict__ t, const RotDev* __restrict__ rots,
                                          int nrot, const typename V2T<R>::type* __restrict__ phase) {
  using V = typename V2T<R>::type;
  constexpr int C = cbinom(W, M);
  V v[C];
  load_beta<V, R>(v, rowp, t, std::make_integer_sequence<int, C>{});
  apply_rots<W, M, REAL, typename V2T<R>::type>(v, rots, nrot);
  store_beta<V, R>(v, rowp, t, phase, std::make_integer_sequence<int, C>{});
}

template <int W, bool REAL, class R, int M = 0>
__device__ __forceinline__ void alpha_m(int m, typename V2T<R>::type* vec, int64_t dim_b, const int* t,
                                        uint32_t col, const RotDev* rots, int nrot,
                                        const typename V2T<R>::type* phase) {
  if constexpr (M <= W) {
    if (m == M)
      alpha_body<W, M, REAL, R>(vec, dim_b, t, col, rots, nrot, phase);
    else
      alpha_m<W, REAL, R, M + 1>(m, vec, dim_b, t, col, rots, nrot, phase);
  }
}

template <int W, bool REAL, class R, int M = 0>
__device__ __forceinline__ void beta_m(int m, typename V2T<R>::type* rowp, const int* t,
                                       const RotDev* rots, int nrot,
                                       const typename V2T<R>::type* phase) {
  if constexpr (M <= W) {
    if (m == M)
      beta_body<W, M, REAL, R>(rowp, t, rots, nrot, phase);
    else
      beta_m<W, REAL, R, M + 1>(m, rowp, t, rots, nrot, phase);
  }
}

template <int W, bool REAL, class R>
__global__ __launch_bounds__(256) void k_win_alpha(typename V2T<R>::type* __restrict__ vec,
                                                   int64_t dim_b, WinDev wt,
                                                   const RotDev* __restrict__ rots, int nrot,
                                                   const typename V2T<R>::type* __restrict__ phase) {
  const int cl = wt.cls[blockIdx.x];
  const int ch = cl >> 6, lane = cl & 63;
  const uint32_t col = blockIdx.y * 256 + threadIdx.x;
  if ((int64_t)col >= dim_b) return;
  const int m = wt.chunk_m[ch];
  // classes with an empty or full window only need touching for a phase
  if (!phase && (m == 0 || m == W)) return;
  const int* t = wt.tab + wt.chunk_off[ch] + lane;
  alpha_m<W, REAL, R>(m, vec, dim_b, t, col, rots, nrot, phase);
}

template <int W, bool REAL, class R>
__global__ __launch_bounds__(256) void k_win_beta(typename V2T<R>::type* __restrict__ vec,
                                                  int64_t dim_a, int64_t dim_b, WinDev wt,
                                                  const RotDev* __restrict__ rots, int nrot,
                                                  const typename V2T<R>::type* __restrict__ phase) {
  const int ch = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.y * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (row >= dim_a) return;
  const int m = wt.chunk_m[ch];
  if (!phase && (m == 0 || m == W)) return;
  const int* t = wt.tab + wt.chunk_off[ch] + lane;
  if (t[0] < 0) return;
  beta_m<W, REAL, R>(m, vec + row * dim_b, t, rots, nrot, phase);
}

template <int W, bool REAL, class R>
static void launch_win(int spin, void* vec, int64_t dim_a, int64_t dim_b, const WinDev& wt,
                       const RotDev* rots, int nrot, const void* phase, hipStream_t s) {
  using V = typename V2T<R>::type;
  if (spin == 0) {
    if (wt.n_cls == 0) return;
    dim3 grid(wt.n_cls, (unsigned)((dim_b + 255) / 256));
    hipLaunchKernelGGL((k_win_alpha<W, REAL, R>), grid, dim3(256), 0, s, (V*)vec, dim_b, wt, rots,
                       nrot, (const V*)phase);
  } else {
    if (wt.n_chunks == 0) return;
    dim3 grid(wt.n_chunks, (unsigned)((dim_a + 3) / 4));
    hipLaunchKernelGGL((k_win_beta<W, REAL, R>), grid, dim3(256), 0, s, (V*)vec, dim_a, dim_b, wt,
                       rots, nrot, (const V*)phase);
  }
}

template <bool REAL, class R>
static void launch_win_w(int spin, void* vec, int64_t dim_a, int64_t dim_b, const WinDev& wt,
                         const RotDev* rots, int nrot, const void* phase, hipStream_t s) {
  switch (wt.w) {
    case 1: launch_win<1, REAL, R>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, s); break;
    case 2: launch_win<2, REAL, R>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, s); break;
    case 3: launch_win<3, REAL, R>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, s); break;
    case 4: launch_win<4, REAL, R>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, s); break;
    case 5: launch_win<5, REAL, R>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, s); break;
    case 6: launch_win<6, REAL, R>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, s); break;
    case 7:
      if constexpr (sizeof(R) == 4) launch_win<7, REAL, R>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, s);
      break;
    default: break;
  }
}

void win_pass(bool c64, bool real, int spin, void* vec, int64_t dim_a, int64_t dim_b,
              const WinDev& wt, const RotDev* rots, int nrot, const void* phase,
              hipStream_t stream) {
  if (c64) {
    if (real)
      launch_win_w<true, float>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, stream);
    else
      launch_win_w<false, float>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, stream);
  } else {
    if (real)
      launch_win_w<true, double>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, stream);
    else
      launch_win_w<false, double>(spin, vec, dim_a, dim_b, wt, rots, nrot, phase, stream);
  }
}

// ---------------------------------------------------------------------------
// per-string tables
// ---------------------------------------------------------------------------
template <class R>
__global__ void k_string_phase(const uint32_t* __restrict__ masks, int64_t n,
                               const double* __restrict__ delta, int norb,
                               typename V2T<R>::type* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t m = masks[i];
  double ang = 0;
  while (m) {
    int p = __builtin_ctz(m);
    ang += delta[p];
    m &= m - 1;
  }
  out[i] = phase_factor<R>(ang);
}

void string_phase(bool c64, const uint32_t* masks, int64_t n, const double* delta, int norb,
                  void* phase, hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256));
  if (c64)
    hipLaunchKernelGGL(k_string_phase<float>, grid, dim3(256), 0, s, masks, n, delta, norb, (zc64*)phase);
  else
    hipLaunchKernelGGL(k_string_phase<double>, grid, dim3(256), 0, s, masks, n, delta, norb, (zc128*)phase);
}

__global__ void k_diag_tables(const uint32_t* __restrict__ ma, int64_t da, const uint32_t* __restrict__ mb,
                              int64_t db, int norb, DiagSpecDev sp, double* __restrict__ A,
                              double* __restrict__ B, double* __restrict__ V) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < da && A) {
    uint32_t m = ma[i];
    double acc = 0;
    for (int p = 0; p < norb; ++p) {
      if (!((m >> p) & 1)) continue;
      if (sp.lin_a) acc += sp.lin_a[p];
      if (sp.Qa)
        for (int q = 0; q < norb; ++q)
          if ((m >> q) & 1) acc += 0.5 * sp.Qa[p * norb + q];
    }
    A[i] = acc;
  }
  if (i < db) {
    uint32_t m = mb[i];
    if (B) {
      double acc = 0;
      for (int p = 0; p < norb; ++p) {
        if (!((m >> p) & 1)) continue;
        if (sp.lin_b) acc += sp.lin_b[p];
        if (sp.Qb)
          for (int q = 0; q < norb; ++q)
            if ((m >> q) & 1) acc += 0.5 * sp.Qb[p * norb + q];
      }
      B[i] = acc;
    }
    if (V && sp.C) {
      for (int p = 0; p < norb; ++p) {
        double acc = 0;
        for (int q = 0; q < norb; ++q)
          if ((m >> q) & 1) acc += sp.C[p * norb + q];
        V[(int64_t)p * db + i] = acc;
      }
    }
  }
}

void diag_tables(const uint32_t* masks_a, int64_t dim_a, const uint32_t* masks_b, int64_t dim_b,
                 int norb, const DiagSpecDev& spec, double* A, double* B, double* V,
                 hipStream_t s) {
  int64_t n = dim_a > dim_b ? dim_a : dim_b;
  hipLaunchKernelGGL(k_diag_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, masks_a, dim_a,
                     masks_b, dim_b, norb, spec, A, B, V);
}

// ---------------------------------------------------------------------------
// diagonal operations: thread <-> column, block <-> (256 columns, ROWS rows)
// ---------------------------------------------------------------------------
constexpr int DIAG_ROWS = 16;

template <int NM>
struct DiagCol {
  double vb[NM];
  double B;
  __device__ __forceinline__ void load(const DiagDev& f, int64_t dim_b, int64_t col, int norb) {
    B = f.B ? f.B[col] : 0.0;
#pragma unroll
    for (int p = 0; p < NM; ++p) vb[p] = (f.V && p < norb) ? f.V[(int64_t)p * dim_b + col] : 0.0;
  }
  __device__ __forceinline__ double eval(const DiagDev& f, int64_t row, uint32_t ma) const {
    double v = B + (f.A ? f.A[row] : 0.0);
    if (f.V) {
#pragma unroll
      for (int p = 0; p < NM; ++p)
        if ((ma >> p) & 1) v += vb[p];
    }
    return v;
  }
};

// mode 0: vec *= exp(i scale f); mode 1: vec *= f
template <int NM, int MODE, class R>
__global__ __launch_bounds__(256) void k_diag_apply(typename V2T<R>::type* __restrict__ vec, int64_t dim_a,
                                                    int64_t dim_b, const uint32_t* __restrict__ masks_a,
                                                    int norb, DiagDev f, double scale) {
  using V = typename V2T<R>::type;
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= dim_b) return;
  DiagCol<NM> dc;
  dc.load(f, dim_b, col, norb);
  const int64_t r0 = (int64_t)blockIdx.y * DIAG_ROWS;
  const int64_t r1 = r0 + DIAG_ROWS < dim_a ? r0 + DIAG_ROWS : dim_a;
  for (int64_t row = r0; row < r1; ++row) {
    double v = dc.eval(f, row, masks_a[row]);
    V x = vec[row * dim_b + col];
    if constexpr (MODE == 0) {
      x = cmul<V, R>(x, phase_factor<R>(scale * v));
    } else {
      x.x *= (R)v;
      x.y *= (R)v;
    }
    vec[row * dim_b + col] = x;
  }
}

template <int NM, class R>
__global__ __launch_bounds__(256) void k_diag_expect(const typename V2T<R>::type* __restrict__ vec,
                                                     int64_t dim_a, int64_t dim_b,
                                                     const uint32_t* __restrict__ masks_a, int norb,
                                                     DiagDev f, double* __restrict__ partials) {
  using V = typename V2T<R>::type;
  __shared__ double sh[4];
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc = 0;
  if (col < dim_b) {
    DiagCol<NM> dc;
    dc.load(f, dim_b, col, norb);
    const int64_t r0 = (int64_t)blockIdx.y * DIAG_ROWS;
    const int64_t r1 = r0 + DIAG_ROWS < dim_a ? r0 + DIAG_ROWS : dim_a;
    for (int64_t row = r0; row < r1; ++row) {
      double v = dc.eval(f, row, masks_a[row]);
      V x = vec[row * dim_b + col];
      acc += v * ((double)x.x * (double)x.x + (double)x.y * (double)x.y);
    }
  }
  double t = block_sum256(acc, sh);
  if (threadIdx.x == 0) partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

static dim3 diag_grid(int64_t dim_a, int64_t dim_b) {
  return dim3((unsigned)((dim_b + 255) / 256), (unsigned)((dim_a + DIAG_ROWS - 1) / DIAG_ROWS));
}

int diag_expect_partials(int64_t dim_a, int64_t dim_b) {
  dim3 g = diag_grid(dim_a, dim_b);
  return (int)(g.x * g.y);
}

template <int MODE, class R>
static void diag_apply_r(void* vec, int64_t da, int64_t db, const uint32_t* ma, int norb,
                         const DiagDev& f, double scale, hipStream_t s) {
  using V = typename V2T<R>::type;
  dim3 g = diag_grid(da, db);
  if (norb <= 16)
    hipLaunchKernelGGL((k_diag_apply<16, MODE, R>), g, dim3(256), 0, s, (V*)vec, da, db, ma, norb, f, scale);
  else
    hipLaunchKernelGGL((k_diag_apply<32, MODE, R>), g, dim3(256), 0, s, (V*)vec, da, db, ma, norb, f, scale);
}

void diag_phase(bool c64, void* vec, int64_t da, int64_t db, const uint32_t* ma, int norb,
                const DiagDev& f, double scale, hipStream_t s) {
  if (c64)
    diag_apply_r<0, float>(vec, da, db, ma, norb, f, scale, s);
  else
    diag_apply_r<0, double>(vec, da, db, ma, norb, f, scale, s);
}

void diag_scale(bool c64, void* vec, int64_t da, int64_t db, const uint32_t* ma, int norb,
                const DiagDev& f, hipStream_t s) {
  if (c64)
    diag_apply_r<1, float>(vec, da, db, ma, norb, f, 0.0, s);
  else
    diag_apply_r<1, double>(vec, da, db, ma, norb, f, 0.0, s);
}

template <class R>
static int diag_expect_r(const void* vec, int64_t da, int64_t db, const uint32_t* ma, int norb,
                         const DiagDev& f, double* partials, hipStream_t s) {
  using V = typename V2T<R>::type;
  dim3 g = diag_grid(da, db);
  if (norb <= 16)
    hipLaunchKernelGGL((k_diag_expect<16, R>), g, dim3(256), 0, s, (const V*)vec, da, db, ma, norb, f, partials);
  else
    hipLaunchKernelGGL((k_diag_expect<32, R>), g, dim3(256), 0, s, (const V*)vec, da, db, ma, norb, f, partials);
  return (int)(g.x * g.y);
}

int diag_expect(bool c64, const void* vec, int64_t da, int64_t db, const uint32_t* ma, int norb,
                const DiagDev& f, double* partials, hipStream_t s) {
  return c64 ? diag_expect_r<float>(vec, da, db, ma, norb, f, partials, s)
             : diag_expect_r<double>(vec, da, db, ma, norb, f, partials, s);
}

// fixed-order sum of n doubles (one block): each thread sums a strided slice,
// then a fixed tree over the block
__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ in, int n, int stride_out,
                                             double* __restrict__ out) {
  __shared__ double sh[4];
  double acc = 0;
  for (int i = threadIdx.x; i < n; i += 256) acc += in[(int64_t)i * stride_out + blockIdx.x];
  double t = block_sum256(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

void sum_partials(const double* partials, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partials, n, 1, out);
}

// <x|y> = sum conj(x) y, partials (re, im) interleaved per block
constexpr int INNER_PER_THREAD = 16;
int inner_partials(int64_t n) { return (int)((n + 256 * INNER_PER_THREAD - 1) / (256 * INNER_PER_THREAD)); }

template <class R>
__global__ __launch_bounds__(256) void k_inner(const typename V2T<R>::type* __restrict__ x,
                                               const typename V2T<R>::type* __restrict__ y, int64_t n,
                                               double* __restrict__ partials) {
  __shared__ double sh[4];
  double re = 0, im = 0;
  const int64_t base = (int64_t)blockIdx.x * 256 * INNER_PER_THREAD + threadIdx.x;
  for (int k = 0; k < INNER_PER_THREAD; ++k) {
    int64_t i = base + (int64_t)k * 256;
    if (i < n) {
      double ax = x[i].x, ay = x[i].y, bx = y[i].x, by = y[i].y;
      re += ax * bx + ay * by;
      im += ax * by - ay * bx;
    }
  }
  double tr = block_sum256(re, sh);
  double ti = block_sum256(im, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = tr;
    partials[2 * blockIdx.x + 1] = ti;
  }
}

void inner(bool c64, const void* x, const void* y, int64_t n, double* partials, double* out,
           hipStream_t s) {
  int nb = inner_partials(n);
  if (c64)
    hipLaunchKernelGGL(k_inner<float>, dim3(nb), dim3(256), 0, s, (const zc64*)x, (const zc64*)y, n, partials);
  else
    hipLaunchKernelGGL(k_inner<double>, dim3(nb), dim3(256), 0, s, (const zc128*)x, (const zc128*)y, n, partials);
  hipLaunchKernelGGL(k_sum, dim3(2), dim3(256), 0, s, partials, nb, 2, out);
}

// ---------------------------------------------------------------------------
// elementwise helpers
// ---------------------------------------------------------------------------
template <class R>
__global__ void k_axpy(const typename V2T<R>::type* __restrict__ x, typename V2T<R>::type* __restrict__ y,
                       int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    auto a = x[i];
    auto b = y[i];
    b.x += a.x;
    b.y += a.y;
    y[i] = b;
  }
}

void axpy(bool c64, const void* x, void* y, int64_t n, hipStream_t s) {
  dim3 g((unsigned)((n + 255) / 256));
  if (c64)
    hipLaunchKernelGGL(k_axpy<float>, g, dim3(256), 0, s, (const zc64*)x, (zc64*)y, n);
  else
    hipLaunchKernelGGL(k_axpy<double>, g, dim3(256), 0, s, (const zc128*)x, (zc128*)y, n);
}

// One step of the Chebyshev recurrence of exp(-i H t) (grid-stride, one
// complex entry per thread and trip):
//   t_next = a * y + b * t_cur + m * t_prev   (stored over t_prev)
//   acc   += coef * t_next
// with y = H t_cur.  Combined in FP64, rounded once to the state's type.
template <class R>
__global__ __launch_bounds__(256) void k_cheb_step(const typename V2T<R>::type* __restrict__ y,
                                                   const typename V2T<R>::type* __restrict__ tcur,
                                                   typename V2T<R>::type* __restrict__ tprev,
                                                   typename V2T<R>::type* __restrict__ acc, int64_t n,
                                                   double a, double b, double m, double cr, double ci) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const auto vy = y[i], vc = tcur[i], va = acc[i];
    double xr = a * (double)vy.x + b * (double)vc.x;
    double xi = a * (double)vy.y + b * (double)vc.y;
    if (m != 0.0) {  // m = 0: t_prev holds no value yet (first step)
      const auto vp = tprev[i];
      xr += m * (double)vp.x;
      xi += m * (double)vp.y;
    }
    typename V2T<R>::type tn, an;
    tn.x = (R)xr;
    tn.y = (R)xi;
    an.x = (R)((double)va.x + (cr * xr - ci * xi));
    an.y = (R)((double)va.y + (cr * xi + ci * xr));
    tprev[i] = tn;
    acc[i] = an;
  }
}

static dim3 stream_grid(int64_t n) {
  const int64_t blocks = (n + 255) / 256;
  return dim3((unsigned)std::min<int64_t>(blocks, 256 * 64));
}

void cheb_step(bool c64, const void* y, const void* tcur, void* tprev, void* acc, int64_t n, double a,
               double b, double m, double cr, double ci, hipStream_t s) {
  if (n <= 0) return;
  if (c64)
    hipLaunchKernelGGL(k_cheb_step<float>, stream_grid(n), dim3(256), 0, s, (const zc64*)y, (const zc64*)tcur,
                       (zc64*)tprev, (zc64*)acc, n, a, b, m, cr, ci);
  else
    hipLaunchKernelGGL(k_cheb_step<double>, stream_grid(n), dim3(256), 0, s, (const zc128*)y,
                       (const zc128*)tcur, (zc128*)tprev, (zc128*)acc, n, a, b, m, cr, ci);
}

// vec *= (cr + i ci)
template <class R>
__global__ __launch_bounds__(256) void k_zscale(typename V2T<R>::type* __restrict__ v, int64_t n, double cr,
                                                double ci) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const auto x = v[i];
    typename V2T<R>::type o;
    o.x = (R)(cr * (double)x.x - ci * (double)x.y);
    o.y = (R)(cr * (double)x.y + ci * (double)x.x);
    v[i] = o;
  }
}

void zscale(bool c64, void* v, int64_t n, double cr, double ci, hipStream_t s) {
  if (n <= 0) return;
  if (c64)
    hipLaunchKernelGGL(k_zscale<float>, stream_grid(n), dim3(256), 0, s, (zc64*)v, n, cr, ci);
  else
    hipLaunchKernelGGL(k_zscale<double>, stream_grid(n), dim3(256), 0, s, (zc128*)v, n, cr, ci);
}

// sum |x - y|^2 in FP64: per-block partials (the blocks of inner()), then a
// fixed-order sum
template <class R>
__global__ __launch_bounds__(256) void k_dist2(const typename V2T<R>::type* __restrict__ x,
                                               const typename V2T<R>::type* __restrict__ y, int64_t n,
                                               double* __restrict__ partials) {
  __shared__ double sh[4];
  double acc = 0;
  const int64_t base = (int64_t)blockIdx.x * 256 * INNER_PER_THREAD + threadIdx.x;
  for (int k = 0; k < INNER_PER_THREAD; ++k) {
    const int64_t i = base + (int64_t)k * 256;
    if (i < n) {
      const double dr = (double)x[i].x - (double)y[i].x, di = (double)x[i].y - (double)y[i].y;
      acc += dr * dr + di * di;
    }
  }
  const double t = block_sum256(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

void dist2(bool c64, const void* x, const void* y, int64_t n, double* partials, double* out, hipStream_t s) {
  const int nb = inner_partials(n);
  if (c64)
    hipLaunchKernelGGL(k_dist2<float>, dim3(nb), dim3(256), 0, s, (const zc64*)x, (const zc64*)y, n, partials);
  else
    hipLaunchKernelGGL(k_dist2<double>, dim3(nb), dim3(256), 0, s, (const zc128*)x, (const zc128*)y, n,
                       partials);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partials, nb, 1, out);
}

// One-body operator of the row spin applied by rows:
//   dst[j, :] = sum_{e in [off[j], off[j+1])} coef[e] * src[srow[e], :]  (+ add[j, :])
// One block per (row j, tile of 2048 columns); the entries of row j are the
// same for the whole block.  FP64 accumulation, one rounding to the state type.
constexpr int kOneBodyPer = 8;
// With dg.A set, the diagonal term w(j, col) src[j, col] is added too, w = A[j] + B[col] +
// sum_{p in row string j} V[p][col] (the tables of a diagonal weight, k_diag_tables).
template <class R>
__global__ __launch_bounds__(256) void k_onebody_rows(const typename V2T<R>::type* __restrict__ src,
                                                      typename V2T<R>::type* dst,
                                                      const typename V2T<R>::type* add, int64_t rows,
                                                      int64_t cols, int64_t tiles, const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ srow,
                                                      const double* __restrict__ coef, OneBodyDiag dg) {
  const int64_t j = (int64_t)blockIdx.x / tiles;
  const int64_t c0 = ((int64_t)blockIdx.x % tiles) * (256 * kOneBodyPer) + threadIdx.x;
  if (j >= rows) return;
  double ar[kOneBodyPer], ai[kOneBodyPer];
#pragma unroll
  for (int k = 0; k < kOneBodyPer; ++k) ar[k] = ai[k] = 0.0;
  const int64_t e1 = off[j + 1];
  for (int64_t e = off[j]; e < e1; ++e) {
    const typename V2T<R>::type* sp = src + (int64_t)srow[e] * cols;
    const double c = coef[e];
#pragma unroll
    for (int k = 0; k < kOneBodyPer; ++k) {
      const int64_t col = c0 + 256 * k;
      if (col < cols) {
        const auto v = sp[col];
        ar[k] += c * (double)v.x;
        ai[k] += c * (double)v.y;
      }
    }
  }
  if (dg.A) {
    const double wa = dg.A[j];
    const uint32_t m = dg.rmasks[j];
#pragma unroll
    for (int k = 0; k < kOneBodyPer; ++k) {
      const int64_t col = c0 + 256 * k;
      if (col < cols) {
        double w = wa + dg.B[col];
        for (int p = 0; p < dg.norb; ++p)
          if ((m >> p) & 1) w += dg.V[(int64_t)p * cols + col];
        const auto v = src[j * cols + col];
        ar[k] += w * (double)v.x;
        ai[k] += w * (double)v.y;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kOneBodyPer; ++k) {
    const int64_t col = c0 + 256 * k;
    if (col < cols) {
      double xr = ar[k], xi = ai[k];
      if (add) {
        const auto a = add[j * cols + col];
        xr += (double)a.x;
        xi += (double)a.y;
      }
      typename V2T<R>::type o;
      o.x = (R)xr;
      o.y = (R)xi;
      dst[j * cols + col] = o;
    }
  }
}

void onebody_rows(bool c64, const void* src, void* dst, const void* add, int64_t rows, int64_t cols,
                  const int64_t* off, const int32_t* srow, const double* coef, const OneBodyDiag& dg, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  const int64_t tiles = (cols + 256 * kOneBodyPer - 1) / (256 * kOneBodyPer);
  const dim3 g((unsigned)(rows * tiles));
  if (c64)
    hipLaunchKernelGGL(k_onebody_rows<float>, g, dim3(256), 0, s, (const zc64*)src, (zc64*)dst, (const zc64*)add,
                       rows, cols, tiles, off, srow, coef, dg);
  else
    hipLaunchKernelGGL(k_onebody_rows<double>, g, dim3(256), 0, s, (const zc128*)src, (zc128*)dst,
                       (const zc128*)add, rows, cols, tiles, off, srow, coef, dg);
}

template <class R>
__global__ void k_outer(const zc128* __restrict__ a, const zc128* __restrict__ b,
                        typename V2T<R>::type* __restrict__ vec, int64_t da, int64_t db) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = blockIdx.y;
  if (col >= db || row >= da) return;
  zc128 x = a[row], y = b[col];
  typename V2T<R>::type r;
  r.x = (R)(x.x * y.x - x.y * y.y);
  r.y = (R)(x.x * y.y + x.y * y.x);
  vec[row * db + col] = r;
}

void outer(bool c64, const double* a, const double* b, void* vec, int64_t da, int64_t db,
           hipStream_t s) {
  dim3 g((unsigned)((db + 255) / 256), (unsigned)da);
  if (c64)
    hipLaunchKernelGGL(k_outer<float>, g, dim3(256), 0, s, (const zc128*)a, (const zc128*)b, (zc64*)vec, da, db);
  else
    hipLaunchKernelGGL(k_outer<double>, g, dim3(256), 0, s, (const zc128*)a, (const zc128*)b, (zc128*)vec, da, db);
}

template <class R>
__global__ __launch_bounds__(256) void k_transpose(const typename V2T<R>::type* __restrict__ src,
                                                   typename V2T<R>::type* __restrict__ dst, int64_t rows,
                                                   int64_t cols) {
  using V = typename V2T<R>::type;
  __shared__ V tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  for (int k = 0; k < 32; k += 8) {
    int64_t r = r0 + ty + k, c = c0 + tx;
    if (r < rows && c < cols) tile[ty + k][tx] = src[r * cols + c];
  }
  __syncthreads();
  for (int k = 0; k < 32; k += 8) {
    int64_t c = c0 + ty + k, r = r0 + tx;
    if (r < rows && c < cols) dst[c * rows + r] = tile[tx][ty + k];
  }
}

void transpose(bool c64, const void* src, void* dst, int64_t rows, int64_t cols, hipStream_t s) {
  dim3 g((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  if (c64)
    hipLaunchKernelGGL(k_transpose<float>, g, dim3(256), 0, s, (const zc64*)src, (zc64*)dst, rows, cols);
  else
    hipLaunchKernelGGL(k_transpose<double>, g, dim3(256), 0, s, (const zc128*)src, (zc128*)dst, rows, cols);
}

// ---------------------------------------------------------------------------
// transition one-body matrix of the row spin
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(256) void k_rdm_rows(const typename V2T<R>::type* __restrict__ lam,
                                                  const typename V2T<R>::type* __restrict__ psi,
                                                  int64_t rows, int64_t cols,
                                                  const uint32_t* __restrict__ masks, int norb,
                                                  double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t i = blockIdx.x;
  const uint32_t I = masks[i];
  const auto* prow = psi + i * cols;
  for (int p = 0; p < norb; ++p) {
    for (int q = 0; q < norb; ++q) {
      double* dst = part + 2 * ((int64_t)(p * norb + q) * rows + i);
      const bool exc = ((I >> q) & 1) && (p == q || !((I >> p) & 1));
      if (!exc) {
        if (threadIdx.x == 0) {
          dst[0] = 0.0;
          dst[1] = 0.0;
        }
        continue;
      }
      uint32_t J = (I & ~(1u << q)) | (1u << p);
      int lo = p < q ? p : q, hi = p < q ? q : p;
      uint32_t between = (hi - lo > 1) ? (I >> (lo + 1)) & ((1u << (hi - lo - 1)) - 1) : 0u;
      const double sign = (__builtin_popcount(between) & 1) ? -1.0 : 1.0;
      const auto* lrow = lam + (int64_t)colex_rank(J) * cols;
      double re = 0, im = 0;
      for (int64_t c = threadIdx.x; c < cols; c += 256) {
        auto a = lrow[c];
        auto b = prow[c];
        double ax = a.x, ay = a.y, bx = b.x, by = b.y;
        re += ax * bx + ay * by;
        im += ax * by - ay * bx;
      }
      double tr = block_sum256(re, sh);
      double ti = block_sum256(im, sh);
      if (threadIdx.x == 0) {
        dst[0] = sign * tr;
        dst[1] = sign * ti;
      }
    }
  }
}

void rdm_rows(bool c64, const void* lam, const void* psi, int64_t rows, int64_t cols,
              const uint32_t* masks_rows, int norb, double* part, hipStream_t s) {
  if (c64)
    hipLaunchKernelGGL(k_rdm_rows<float>, dim3((unsigned)rows), dim3(256), 0, s, (const zc64*)lam,
                       (const zc64*)psi, rows, cols, masks_rows, norb, part);
  else
    hipLaunchKernelGGL(k_rdm_rows<double>, dim3((unsigned)rows), dim3(256), 0, s, (const zc128*)lam,
                       (const zc128*)psi, rows, cols, masks_rows, norb, part);
}

// Transition one-body matrix of the column spin through the strings K of one
// electron fewer: for K and orbitals p, q outside it, lam's string K + p and
// psi's string K + q contribute conj(lam) psi s_p(K) s_q(K) to T_pq.  Over K
// this is a product of a 16 x |K| by a |K| x 16 matrix whose entries are
// zero for orbitals inside K, so it runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]
// and receives D[l / 16 + 4 t][l % 16], t = 0..3).  Each lane gathers one
// amplitude of lam and one of psi for (orbital l % 16, string l / 16) of a
// block of four strings; the real and imaginary parts take four products in
// four independent accumulators.  One block per row; the groups of K are
// taken in turn with their home columns and string list staged in LDS.  The
// sums run in a fixed order (per wave over its string blocks, then over the
// waves in order).
typedef double rdm_d4 __attribute__((ext_vector_type(4)));
constexpr int kRdmMfmaThreads = 1024;

template <class R>
__global__ __launch_bounds__(kRdmMfmaThreads) void k_rdm_mfma(RdmMfmaDev P) {
  using V = typename V2T<R>::type;
  extern __shared__ __align__(16) char smem[];
  V* hl = (V*)smem;                                    // lam, home columns
  V* hp = hl + P.max_home;                             // psi, home columns
  uint32_t* kl = (uint32_t*)(hp + P.max_home);         // the group's strings K
  __shared__ int rlo[256];
  __shared__ int rhi[256 * 17];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  const int64_t row = blockIdx.x;
  for (int i = tid; i < 256; i += nthr) rlo[i] = P.rank_lo[i];
  for (int i = tid; i < 256 * 17; i += nthr) rhi[i] = P.rank_hi[i];
  const V* lr = (const V*)P.lam + row * P.cols;
  const V* pr = (const V*)P.psi + row * P.cols;
  const int o = lane & 15, kk = lane >> 4;
  const bool o_in = o < P.norb, o_home = o < P.nlow;
  const uint32_t below = (1u << o) - 1u;
  rdm_d4 rr = {0.0, 0.0, 0.0, 0.0}, ii = rr, ri = rr, ir = rr;
  for (int g = 0; g < P.ngroups; ++g) {
    const int4 gd = uniform_load((const int4*)P.group + g);  // home_off, home_len, first K, count
    __syncthreads();
    for (int e0 = tid; e0 < gd.y; e0 += 4 * nthr) {
      V a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * nthr, gd.y - 1);
        a[u] = lr[gd.x + e];
        b[u] = pr[gd.x + e];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        keep(a[u]);
        keep(b[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * nthr < gd.y) {
          hl[e0 + u * nthr] = a[u];
          hp[e0 + u * nthr] = b[u];
        }
    }
    for (int e = tid; e < gd.w; e += nthr) kl[e] = P.inter[gd.z + e];
    __syncthreads();
    const int nkb = (gd.w + 3) >> 2;
    for (int kb = wave; kb < nkb; kb += nw) {
      const int k = 4 * kb + kk;
      double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
      if (k < gd.w && o_in) {
        const uint32_t K = kl[k];
        if (!((K >> o) & 1u)) {
          const uint32_t J = K | (1u << o);
          const int rk = rlo[J & 255u] + rhi[(J >> 8) * 17 + __builtin_popcount(J & 255u)];
          V a, b;
          if (o_home) {
            a = hl[rk - gd.x];
            b = hp[rk - gd.x];
          } else {
            a = lr[rk];
            b = pr[rk];
          }
          ar = (double)a.x;
          ai = (double)a.y;
          br = (double)b.x;
          bi = (double)b.y;
          if (__builtin_popcount(K & below) & 1) {
            ar = -ar;
            ai = -ai;
            br = -br;
            bi = -bi;
          }
        }
      }
      // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
      rr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, rr, 0, 0, 0);
      ii = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, ii, 0, 0, 0);
      ri = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, ri, 0, 0, 0);
      ir = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, ir, 0, 0, 0);
    }
  }
  __syncthreads();
  double* red = (double*)smem;  // [wave][re 256 | im 256]
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int pq = (kk + 4 * t) * 16 + o;
    red[wave * 512 + pq] = rr[t] + ii[t];
    red[wave * 512 + 256 + pq] = ri[t] - ir[t];
  }
  __syncthreads();
  const int nn = P.norb * P.norb;
  for (int i = tid; i < nn; i += nthr) {
    const int p = i / P.norb, q = i - p * P.norb;
    double re = 0.0, im = 0.0;
    for (int w = 0; w < nw; ++w) {
      re += red[w * 512 + p * 16 + q];
      im += red[w * 512 + 256 + p * 16 + q];
    }
    P.part[2 * ((int64_t)i * P.rows + row)] = re;
    P.part[2 * ((int64_t)i * P.rows + row) + 1] = im;
  }
}

size_t rdm_mfma_lds(bool c64, int max_home, int max_inter) {
  const size_t home = 2 * (size_t)max_home * (c64 ? 8 : 16) + (size_t)max_inter * 4;
  const size_t red = (size_t)(kRdmMfmaThreads / 64) * 512 * 8;
  return std::max(home, red);
}

void rdm_mfma(bool c64, const RdmMfmaDev& d, hipStream_t s) {
  const size_t lds = rdm_mfma_lds(c64, d.max_home, d.max_inter);
  if (c64) {
    static bool set = false;
    if (!set) {
      (void)hipFuncSetAttribute((const void*)k_rdm_mfma<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024 - 20 * 1024);
      (void)hipGetLastError();
      set = true;
    }
    hipLaunchKernelGGL(k_rdm_mfma<float>, dim3((unsigned)d.rows), dim3(kRdmMfmaThreads), lds, s, d);
  } else {
    static bool set = false;
    if (!set) {
      (void)hipFuncSetAttribute((const void*)k_rdm_mfma<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024 - 20 * 1024);
      (void)hipGetLastError();
      set = true;
    }
    hipLaunchKernelGGL(k_rdm_mfma<double>, dim3((unsigned)d.rows), dim3(kRdmMfmaThreads), lds, s, d);
  }
}

__global__ __launch_bounds__(256) void k_rdm_reduce(const double* __restrict__ part, int64_t rows,
                                                    double* __restrict__ T) {
  __shared__ double sh[4];
  const int64_t pq = blockIdx.x;
  double re = 0, im = 0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) {
    re += part[2 * (pq * rows + i)];
    im += part[2 * (pq * rows + i) + 1];
  }
  double tr = block_sum256(re, sh);
  double ti = block_sum256(im, sh);
  if (threadIdx.x == 0) {
    T[2 * pq] = tr;
    T[2 * pq + 1] = ti;
  }
}

void rdm_reduce(const double* part, int64_t rows, int norb, double* T, hipStream_t s) {
  hipLaunchKernelGGL(k_rdm_reduce, dim3(norb * norb), dim3(256), 0, s, part, rows, T);
}

// ---------------------------------------------------------------------------
// diagonal-gate gradient reductions
// ---------------------------------------------------------------------------
template <int NM, class R>
__global__ __launch_bounds__(256) void k_diag_grad_rows(const typename V2T<R>::type* __restrict__ lam,
                                                        const typename V2T<R>::type* __restrict__ psi,
                                                        int64_t dim_a, int64_t dim_b,
                                                        const uint32_t* __restrict__ masks_b, int norb,
                                                        double* __restrict__ rowout) {
  __shared__ double sh[4];
  const int64_t row = blockIdx.x;
  double acc[2 * NM];
#pragma unroll
  for (int k = 0; k < 2 * NM; ++k) acc[k] = 0;
  for (int64_t c = threadIdx.x; c < dim_b; c += 256) {
    auto a = lam[row * dim_b + c];
    auto b = psi[row * dim_b + c];
    double z = (double)a.x * (double)b.y - (double)a.y * (double)b.x;
    uint32_t m = masks_b[c];
    acc[0] += z;
#pragma unroll
    for (int p = 0; p < NM; ++p) {
      double bp = (double)((m >> p) & 1);
      acc[1 + p] += z * bp;
      if (p + 1 < NM) acc[1 + NM + p] += z * bp * (double)((m >> (p + 1)) & 1);
    }
  }
  // layout per row: [0] = 1, [1 + p] = x_b[p], [1 + norb + p] = x_b[p] x_b[p+1]
#pragma unroll
  for (int k = 0; k < 2 * NM; ++k) {
    double t = block_sum256(acc[k], sh);
    if (threadIdx.x == 0) {
      if (k == 0) rowout[row * 2 * norb] = t;
      else if (k <= NM) {
        int p = k - 1;
        if (p < norb) rowout[row * 2 * norb + 1 + p] = t;
      } else {
        int p = k - 1 - NM;
        if (p < norb - 1) rowout[row * 2 * norb + 1 + norb + p] = t;
      }
    }
  }
}

void diag_grad_rows(bool c64, const void* lam, const void* psi, int64_t da, int64_t db,
                    const uint32_t* masks_b, int norb, double* rowout, hipStream_t s) {
  if (c64) {
    if (norb <= 16)
      hipLaunchKernelGGL((k_diag_grad_rows<16, float>), dim3((unsigned)da), dim3(256), 0, s, (const zc64*)lam,
                         (const zc64*)psi, da, db, masks_b, norb, rowout);
    else
      hipLaunchKernelGGL((k_diag_grad_rows<32, float>), dim3((unsigned)da), dim3(256), 0, s, (const zc64*)lam,
                         (const zc64*)psi, da, db, masks_b, norb, rowout);
  } else {
    if (norb <= 16)
      hipLaunchKernelGGL((k_diag_grad_rows<16, double>), dim3((unsigned)da), dim3(256), 0, s, (const zc128*)lam,
                         (const zc128*)psi, da, db, masks_b, norb, rowout);
    else
      hipLaunchKernelGGL((k_diag_grad_rows<32, double>), dim3((unsigned)da), dim3(256), 0, s, (const zc128*)lam,
                         (const zc128*)psi, da, db, masks_b, norb, rowout);
  }
}

// ---------------------------------------------------------------------------
// gradient of a diagonal Coulomb gate with respect to its matrix: per alpha
// row i_a, out[p * norb + q] = sum_{i_b} Im(conj(lam) psi) x_p x_q with
// x = x_a + x_b the total occupation; thread t owns the pair t, column blocks
// of z and of the beta masks are staged in LDS
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(256) void k_dc_grad_rows(const typename V2T<R>::type* __restrict__ lam,
                                                      const typename V2T<R>::type* __restrict__ psi,
                                                      int64_t dim_a, int64_t dim_b,
                                                      const uint32_t* __restrict__ masks_a,
                                                      const uint32_t* __restrict__ masks_b, int norb,
                                                      double* __restrict__ rowout) {
  constexpr int CH = 2048;
  __shared__ double z[CH];
  __shared__ uint32_t mk[CH];
  const int64_t row = blockIdx.x;
  const uint32_t xa = masks_a[row];
  const int NN = norb * norb;
  for (int t0 = 0; t0 < NN; t0 += 256) {
    const int t = t0 + (int)threadIdx.x;
    const int p = t / norb, q = t - (t / norb) * norb;
    const double ap = t < NN ? (double)((xa >> p) & 1) : 0.0;
    const double aq = t < NN ? (double)((xa >> q) & 1) : 0.0;
    double acc = 0.0;
    for (int64_t c0 = 0; c0 < dim_b; c0 += CH) {
      const int n = (int)(dim_b - c0 < CH ? dim_b - c0 : CH);
      __syncthreads();
      for (int e = threadIdx.x; e < n; e += 256) {
        const auto a = lam[row * dim_b + c0 + e];
        const auto b = psi[row * dim_b + c0 + e];
        z[e] = (double)a.x * (double)b.y - (double)a.y * (double)b.x;
        mk[e] = masks_b[c0 + e];
      }
      __syncthreads();
      if (t < NN)
        for (int e = 0; e < n; ++e) {
          const uint32_t w = mk[e];
          acc += z[e] * (ap + (double)((w >> p) & 1)) * (aq + (double)((w >> q) & 1));
        }
    }
    if (t < NN) rowout[row * NN + t] = acc;
  }
}

void dc_grad_rows(bool c64, const void* lam, const void* psi, int64_t da, int64_t db, const uint32_t* masks_a,
                  const uint32_t* masks_b, int norb, double* rowout, hipStream_t s) {
  if (c64)
    hipLaunchKernelGGL(k_dc_grad_rows<float>, dim3((unsigned)da), dim3(256), 0, s, (const zc64*)lam,
                       (const zc64*)psi, da, db, masks_a, masks_b, norb, rowout);
  else
    hipLaunchKernelGGL(k_dc_grad_rows<double>, dim3((unsigned)da), dim3(256), 0, s, (const zc128*)lam,
                       (const zc128*)psi, da, db, masks_a, masks_b, norb, rowout);
}

void sum_columns(const double* in, int rows, int width, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3((unsigned)width), dim3(256), 0, s, in, rows, width, out);
}

__global__ __launch_bounds__(256) void k_diag_grad_combine(const double* __restrict__ rowout, int64_t dim_a,
                                                           const uint32_t* __restrict__ masks_a, int norb,
                                                           double* __restrict__ out) {
  __shared__ double sh[4];
  const int k = blockIdx.x;  // 0 .. 2 norb - 2
  double acc = 0;
  for (int64_t i = threadIdx.x; i < dim_a; i += 256) {
    uint32_t m = masks_a[i];
    const double* r = rowout + i * 2 * norb;
    if (k < norb - 1) {
      int p = k;
      double both = (double)(((m >> p) & 1) & ((m >> (p + 1)) & 1));
      acc += both * r[0] + r[1 + norb + p];
    } else {
      int p = k - (norb - 1);
      acc += (double)((m >> p) & 1) * r[1 + p];
    }
  }
  double t = block_sum256(acc, sh);
  if (threadIdx.x == 0) out[k] = 2.0 * t;
}

void diag_grad_combine(const double* rowout, int64_t dim_a, const uint32_t* masks_a, int norb,
                       double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_grad_combine, dim3(2 * norb - 1), dim3(256), 0, s, rowout, dim_a, masks_a,
                     norb, out);
}

}  // namespace dev
}  // namespace ffx
