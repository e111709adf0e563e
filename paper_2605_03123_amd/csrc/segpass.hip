// Segment passes (gfx950): every Givens rotation and diagonal gate that acts
// on the column strings of one row of the state, applied with one HBM round
// trip of that row.
//
// The state is read row-wise (for the alpha-major matrix Gamma the column
// strings are the beta configurations; for its transpose they are the alpha
// configurations).  Rotations of the column spin never mix rows (Sec. 3.2.3:
// a Givens rotation of spin sigma pairs configurations that differ only in
// spin sigma), so a block can load a whole row -- or a contiguous segment of
// it whose configurations share the occupation of the orbitals above the
// segment window -- into LDS and run a list of stages on it:
//   * Givens stages: rotations confined to a register window [a, a+W); each
//     lane loads one class of configurations that agree outside the window
//     from LDS into registers, applies the stage's rotations there, and writes
//     the class back (one LDS round trip per stage, never per rotation);
//   * diagonal stages: per-configuration phases (number-operator sums,
//     diagonal Coulomb, deferred orbital phase layers), weights or weighted
//     norms, evaluated in FP64 from the row string, the column string and
//     byte-indexed partial-sum tables kept in LDS.
// The row segment is then stored once (or accumulated, or dropped after a
// reduction).
#include <hip/hip_runtime.h>

#include <utility>

#include "dev_common.h"
#include "device.h"

namespace ffx {
namespace dev {

template <int W, int M, bool REAL, class R, int... K>
__device__ __forceinline__ void lds_class(typename V2T<R>::type* __restrict__ row, const int* __restrict__ t,
                                          const RotDev* __restrict__ rots, int nrot,
                                          std::integer_sequence<int, K...>) {
  using V = typename V2T<R>::type;
  V v[sizeof...(K)];
  ((v[K] = row[t[K * 64]]), ...);
  apply_rots<W, M, REAL, R>(v, rots, nrot);
  const volatile int* tv = t;
  ((row[tv[K * 64]] = v[K]), ...);
}

template <int W, bool REAL, class R, int M = 1>
__device__ __forceinline__ void lds_m(int m, typename V2T<R>::type* row, const int* t, const RotDev* rots,
                                      int nrot) {
  if constexpr (M < W) {
    if (m == M)
      lds_class<W, M, REAL, R>(row, t, rots, nrot, std::make_integer_sequence<int, cbinom(W, M)>{});
    else
      lds_m<W, REAL, R, M + 1>(m, row, t, rots, nrot);
  }
}

__device__ __forceinline__ int parity(uint32_t x) { return __builtin_popcount(x) & 1; }

template <int W, bool REAL, class R>
__global__ __launch_bounds__(768) void k_seg_pass(SegPassDev P) {
  using V = typename V2T<R>::type;
  extern __shared__ __align__(16) char smem[];
  V* row = (V*)smem;
  double* tab = (double*)(smem + P.lds_row_bytes);  // 4 x 256 byte tables
  double* wq = tab + 4 * 256;                       // 32 cross weights
  double* red = wq + 32;                            // block reduction scratch

  const int64_t blk = blockIdx.x;
  const int si = (int)(blk % P.n_seg);
  const int64_t r = blk / P.n_seg;
  const SegDev sg = P.segs[si];
  const int nthr = blockDim.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nwaves = nthr >> 6;

  const V* src = (const V*)P.src + r * P.row_len + sg.off;
  for (int e = tid; e < sg.len; e += nthr) row[e] = src[e];
  __syncthreads();

  const uint32_t rmask = P.row_masks[r];
  const uint32_t* cmask = P.col_masks + sg.off;
  const int nbytes = (P.norb + 7) >> 3;
  double acc = 0.0;

  for (int s = 0; s < P.n_stages; ++s) {
    const StageDev st = P.stages[s];
    if (st.type == ST_GIVENS) {
      const WinDev wt = sg.win[st.a];
      for (int ch = wave; ch < wt.n_chunks; ch += nwaves) {
        const int m = wt.chunk_m[ch];
        if (m == 0 || m == W) continue;
        const int* t = wt.tab + wt.chunk_off[ch] + lane;
        if (t[0] >= 0) lds_m<W, REAL, R>(m, row, t, st.rots, st.nrot);
      }
    } else {
      // cross weights w[q] = sum_{p in row} C[p][q]
      const double coef = (st.type == ST_PHASE) ? st.scale : 1.0;
      if (tid < P.norb) {
        double w = 0.0;
        if (st.C)
          for (int p = 0; p < P.norb; ++p)
            if ((rmask >> p) & 1) w += st.C[p * P.norb + tid];
        w *= coef;
        if (st.type == ST_PHASE && st.dcol) w += st.dcol[tid];
        wq[tid] = w;
      }
      __syncthreads();
      for (int i = tid; i < nbytes * 256; i += nthr) {
        const int k = i >> 8, b = i & 255;
        double v = 0.0;
        for (int q = 0; q < 8; ++q)
          if (((b >> q) & 1) && 8 * k + q < P.norb) v += wq[8 * k + q];
        tab[i] = v;
      }
      __syncthreads();
      double arow = st.A ? st.A[r] : 0.0;
      double grow = 0.0;
      if (st.type == ST_PHASE && st.drow)
        for (int p = 0; p < P.norb; ++p)
          if ((rmask >> p) & 1) grow += st.drow[p];
      const int srow = parity(rmask & st.sign_row);
      for (int e = tid; e < sg.len; e += nthr) {
        const uint32_t cm = cmask[e];
        double x = 0.0;
        for (int k = 0; k < nbytes; ++k) x += tab[(k << 8) | ((cm >> (8 * k)) & 255)];
        const double bcol = st.B ? st.B[sg.off + e] : 0.0;
        V y = row[e];
        if (st.type == ST_PHASE) {
          const double ang = st.scale * (arow + bcol) + x + grow;
          V ph = phase_factor<R>(ang);
          if (srow ^ parity(cm & st.sign_col)) {
            ph.x = -ph.x;
            ph.y = -ph.y;
          }
          row[e] = cmul<V, R>(y, ph);
        } else {
          const double f = arow + bcol + x;
          if (st.type == ST_SCALE) {
            y.x = (R)(f * (double)y.x);
            y.y = (R)(f * (double)y.y);
            row[e] = y;
          } else {
            acc += f * ((double)y.x * (double)y.x + (double)y.y * (double)y.y);
          }
        }
      }
    }
    __syncthreads();
  }

  if (P.mode != SEG_NONE) {
    V* dst = (V*)P.dst + r * P.row_len + sg.off;
    if (P.mode == SEG_STORE) {
      for (int e = tid; e < sg.len; e += nthr) dst[e] = row[e];
    } else {
      for (int e = tid; e < sg.len; e += nthr) {
        V a = dst[e], b = row[e];
        a.x += b.x;
        a.y += b.y;
        dst[e] = a;
      }
    }
  }
  if (P.partials) {
    // fixed-order block reduction: wave sums, then wave 0 adds them in order
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int i = 0; i < nwaves; ++i) t += red[i];
      P.partials[blk] = t;
    }
  }
}

size_t seg_pass_lds(bool c64, int max_len) {
  size_t row = (size_t)max_len * (c64 ? 8 : 16);
  row = (row + 15) & ~(size_t)15;
  return row + (4 * 256 + 32 + 16) * sizeof(double);
}

template <int W, bool REAL, class R>
static void launch_seg(const SegPassDev& p, int threads, size_t lds, hipStream_t s) {
  auto k = k_seg_pass<W, REAL, R>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  const int64_t blocks = p.n_rows * p.n_seg;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(threads), lds, s, p);
}

template <bool REAL, class R>
static void launch_seg_w(int W, const SegPassDev& p, int threads, size_t lds, hipStream_t s) {
  switch (W) {
    case 1: launch_seg<1, REAL, R>(p, threads, lds, s); break;
    case 2: launch_seg<2, REAL, R>(p, threads, lds, s); break;
    case 3: launch_seg<3, REAL, R>(p, threads, lds, s); break;
    case 4: launch_seg<4, REAL, R>(p, threads, lds, s); break;
    case 5: launch_seg<5, REAL, R>(p, threads, lds, s); break;
    case 6: launch_seg<6, REAL, R>(p, threads, lds, s); break;
    case 7:
      if constexpr (sizeof(R) == 4) launch_seg<7, REAL, R>(p, threads, lds, s);
      break;
    default: break;
  }
}

void seg_pass(bool c64, bool real, int W, const SegPassDev& p, int threads, size_t lds, hipStream_t s) {
  if (c64) {
    if (real)
      launch_seg_w<true, float>(W, p, threads, lds, s);
    else
      launch_seg_w<false, float>(W, p, threads, lds, s);
  } else {
    if (real)
      launch_seg_w<true, double>(W, p, threads, lds, s);
    else
      launch_seg_w<false, double>(W, p, threads, lds, s);
  }
}

// ---------------------------------------------------------------------------
// in-place transpose of a square matrix: block (bx, by) with bx <= by swaps
// tile (by, bx) with tile (bx, by) through LDS (a diagonal tile is transposed
// in place).
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(256) void k_transpose_square(typename V2T<R>::type* __restrict__ a, int64_t n,
                                                          int64_t ntiles) {
  using V = typename V2T<R>::type;
  __shared__ V t0[32][33];
  __shared__ V t1[32][33];
  // map the linear block index onto the lower triangle (bx <= by) of tile pairs
  int64_t k = blockIdx.x;
  int64_t by = (int64_t)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
  while ((by + 1) * (by + 2) / 2 <= k) ++by;
  while (by * (by + 1) / 2 > k) --by;
  const int64_t bx = k - by * (by + 1) / 2;
  if (by >= ntiles) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t r0 = by * 32, c0 = bx * 32;  // tile (by, bx)
  for (int j = ty; j < 32; j += 8) {
    int64_t r = r0 + j, c = c0 + tx;
    if (r < n && c < n) t0[j][tx] = a[r * n + c];
    int64_t r2 = c0 + j, c2 = r0 + tx;  // tile (bx, by)
    if (r2 < n && c2 < n) t1[j][tx] = a[r2 * n + c2];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    // tile (bx, by) <- transpose of tile (by, bx), and vice versa
    int64_t r2 = c0 + j, c2 = r0 + tx;
    if (r2 < n && c2 < n) a[r2 * n + c2] = t0[tx][j];
    int64_t r = r0 + j, c = c0 + tx;
    if (r < n && c < n) a[r * n + c] = t1[tx][j];
  }
}

void transpose_square(bool c64, void* vec, int64_t n, hipStream_t s) {
  const int64_t nt = (n + 31) / 32;
  const int64_t blocks = nt * (nt + 1) / 2;
  if (c64)
    hipLaunchKernelGGL(k_transpose_square<float>, dim3((unsigned)blocks), dim3(256), 0, s, (zc64*)vec, n, nt);
  else
    hipLaunchKernelGGL(k_transpose_square<double>, dim3((unsigned)blocks), dim3(256), 0, s, (zc128*)vec, n, nt);
}

}  // namespace dev
}  // namespace ffx
