// Batched execution (gfx950): many independent sectors of uneven size, each
// running its own list of passes (LUCJ forward, costate, energy, reverse sweep
// with transition one-body matrices), run together.
//
// A task is a block of consecutive rows (or of consecutive columns: the rows
// of the transposed layout) of one instance's state, or a small per-instance
// job (tables, fixed-order sums).  Pass k of every instance forms level k; the
// passes of one level never depend on each other.
//
// k_batch_coop runs the whole batch as one cooperative launch with a grid
// barrier between levels; k_batch_kind runs one level's tasks of one kind per
// launch, one block per task.  k_batch is the single persistent launch over
// the same queue:
// blocks take tasks with an atomic counter and wait, before each task, until
// every task of the same instance's earlier passes has finished
// (per-instance counters, relaxed polling with sleeps, one agent-scope
// acquire per task, a wall-clock bound after which every block leaves).  It is
// built but not launched: its runs on the GPU did not complete and the cause
// is not established.
//
// Givens and diagonal stages run on the task's rows held back to back in LDS,
// with the class tables of one row replicated over the rows (see
// replicate_seg_window), so small rows still fill the 64 lanes of a wave.
// Columns are gathered and scattered directly, so no transposes are needed.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "dev_common.h"
#include "device.h"

namespace ffx {
namespace dev {

constexpr int kBatchThreads = 256;
typedef double bdouble4 __attribute__((ext_vector_type(4)));
typedef double bdouble2 __attribute__((ext_vector_type(2)));
typedef float bfloat2 __attribute__((ext_vector_type(2)));
constexpr int kBatchMaxRows = 64;   // rows per task
constexpr int kBatchMaxOrb = 16;    // orbitals of a batched sector
// bounded wait, in ticks of the 100 MHz real-time counter (2 s)
constexpr uint64_t kWaitTicks = 200000000ull;
// dynamic LDS limit: the kernel's own static LDS (a few scalars) shares the 160 KB
constexpr int kBatchMaxDynLds = 160 * 1024 - 256;

struct BatchLds {
  char* rows;
  int* mt;
  double* wq;      // wq_rows x kBatchMaxOrb cross weights
  double* rowf;    // wq_rows complex row factors (or real row values)
  double* acc;     // 4 waves x 2 N^2 doubles (RDM) or 4 x 2N (diagonal gradients)
  double* red;     // 16 doubles
};

// LDS of a block: the rows, then red (16 doubles), then either the segment
// tables (mt, wq, rowf: segment tasks) or acc (the other kinds).  A launch
// that runs one kind allocates only that kind's part; the all-kinds kernels
// lay both out, the tables first (kind = -1).
constexpr int kRedDoubles = 16;
constexpr int kAccDoubles = 4 * 2 * kBatchMaxOrb * kBatchMaxOrb;
// doubles of the cross weights and row factors of a task of at most wq_rows rows
__host__ __device__ inline size_t seg_tab_doubles(int wq_rows) {
  return (size_t)wq_rows * kBatchMaxOrb + 2 * (size_t)wq_rows;
}

__host__ __device__ inline size_t batch_lds_kind(int kind, int lds_row_bytes, int max_mt, int wq_rows) {
  const size_t tabs = (size_t)((max_mt + 3) & ~3) * 4 + seg_tab_doubles(wq_rows) * 8;
  const size_t head = (size_t)lds_row_bytes + (size_t)kRedDoubles * 8;
  if (kind == BK_SEG) return head + tabs;
  if (kind >= 0) return head + (size_t)kAccDoubles * 8;
  return head + tabs + (size_t)kAccDoubles * 8;
}

__device__ __forceinline__ BatchLds batch_lds_map(char* smem, const BatchDev& B, int kind = -1) {
  BatchLds L{};
  L.rows = smem;
  L.red = (double*)(smem + B.lds_row_bytes);
  char* p = (char*)(L.red + kRedDoubles);
  if (kind == BK_SEG || kind < 0) {
    L.mt = (int*)p;
    L.wq = (double*)(L.mt + ((B.max_mt + 3) & ~3));
    L.rowf = L.wq + B.wq_rows * kBatchMaxOrb;
    p = (char*)(L.rowf + 2 * B.wq_rows);
  }
  if (kind != BK_SEG) L.acc = (double*)p;
  return L;
}

size_t batch_lds(bool c64, int lds_row_bytes, int max_mt, int wq_rows) {
  (void)c64;
  return batch_lds_kind(-1, lds_row_bytes, max_mt, wq_rows);
}

size_t batch_lds_for(int kind, int lds_row_bytes, int max_mt, int wq_rows) {
  return batch_lds_kind(kind, lds_row_bytes, max_mt, wq_rows);
}

// fixed-order block sum (4 waves); every thread gets the result
__device__ __forceinline__ double batch_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = red[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  __syncthreads();
  return t;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// a two-entry field picked by a runtime index without indexing into the struct
// (which would move the struct to scratch memory)
template <class T>
__device__ __forceinline__ T pick2(const T (&a)[2], int i) {
  return i ? a[1] : a[0];
}

// element k of row r of the layout (0: alpha-major rows, 1: columns)
__device__ __forceinline__ int64_t lay_index(int layout, int64_t r, int64_t k, int64_t ncols_state) {
  return layout == 0 ? r * ncols_state + k : k * ncols_state + r;
}

// ---------------------------------------------------------------------------
// tables of a program: per-string diagonal values and column phase factors
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tables_task(const BPassDev& ps, const BTypeDev& ty, int task) {
  const BTableDev e = uniform_load(ps.tables + task);
  const int N = ty.norb;
  if (e.kind == 0) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      double* out = s == 0 ? e.A : e.B;
      if (!out) continue;
      const double* lin = s == 0 ? e.spec.lin_a : e.spec.lin_b;
      const double* Q = s == 0 ? e.spec.Qa : e.spec.Qb;
      for (int64_t i = threadIdx.x; i < ty.dim[s]; i += blockDim.x) {
        const uint32_t m = ty.masks[s][i];
        double acc = 0;
        for (int p = 0; p < N; ++p) {
          if (!((m >> p) & 1)) continue;
          if (lin) acc += lin[p];
          if (Q)
            for (int q = 0; q < N; ++q)
              if ((m >> q) & 1) acc += 0.5 * Q[p * N + q];
        }
        out[i] = acc;
      }
    }
  } else {
    zc128* out = (zc128*)e.out;
    for (int64_t i = threadIdx.x; i < pick2(ty.dim, e.spin); i += blockDim.x) {
      const uint32_t m = pick2(ty.masks, e.spin)[i];
      double ang = e.cB ? e.scale * e.cB[i] : 0.0;
      if (e.delta)
        for (uint32_t x = m; x; x &= x - 1) ang += e.delta[__builtin_ctz(x)];
      zc128 f = phase_factor<double>(ang);
      if (__builtin_popcount(m & e.sign) & 1) {
        f.x = -f.x;
        f.y = -f.y;
      }
      out[i] = f;
    }
  }
}

// ---------------------------------------------------------------------------
// Slater outer product, inner product, fixed-order sums
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void outer_task(const BPassDev& ps, const BTypeDev& ty, int task) {
  using V = typename V2T<R>::type;
  const int RR = ty.rows_per_task[1];
  const int64_t db = ty.dim[1];
  const int64_t r0 = (int64_t)task * RR;
  const int64_t n = std::min<int64_t>(RR, ty.dim[0] - r0) * db;
  const zc128* a = (const zc128*)ps.oa + r0;
  const zc128* b = (const zc128*)ps.ob;
  V* out = (V*)ps.dst + r0 * db;
  for (int64_t x = threadIdx.x; x < n; x += blockDim.x) {
    const zc128 u = a[x / db], v = b[x % db];
    V o;
    o.x = (R)(u.x * v.x - u.y * v.y);
    o.y = (R)(u.x * v.y + u.y * v.x);
    out[x] = o;
  }
}

template <class R>
__device__ __forceinline__ void inner_task(const BPassDev& ps, const BTypeDev& ty, int task, double* red) {
  using V = typename V2T<R>::type;
  const int RR = ty.rows_per_task[1];
  const int64_t db = ty.dim[1];
  const int64_t r0 = (int64_t)task * RR;
  const int64_t n = std::min<int64_t>(RR, ty.dim[0] - r0) * db;
  const V* x = (const V*)ps.src + r0 * db;
  const V* y = (const V*)ps.src2 + r0 * db;
  double re = 0, im = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double ax = x[i].x, ay = x[i].y, bx = y[i].x, by = y[i].y;
    re += ax * bx + ay * by;
    im += ax * by - ay * bx;
  }
  re = batch_block_sum(re, red);
  im = batch_block_sum(im, red);
  if (threadIdx.x == 0) {
    ps.partials[2 * task] = re;
    ps.partials[2 * task + 1] = im;
  }
}

__device__ __forceinline__ void sum_task(const BPassDev& ps) {
  // partials are requested 16 at a time and added in index order, so the sum
  // is the same as one term at a time but waits on one memory latency per 16
  constexpr int U = 16;
  for (int w = threadIdx.x; w < ps.width; w += blockDim.x) {
    const double* p = ps.partials + w;
    double t = 0;
    int k = 0;
    for (; k + U <= ps.n_sum; k += U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = p[(int64_t)(k + u) * ps.width];
#pragma unroll
      for (int u = 0; u < U; ++u) t += v[u];
    }
    for (; k < ps.n_sum; ++k) t += p[(int64_t)k * ps.width];
    ps.out[w] = t;
  }
}

// ---------------------------------------------------------------------------
// transition one-body matrix of the column spin of a layout, from a block of
// rows (or columns) of lam and psi staged in LDS:
//   T[p][q] = sum_rows sum_{I -> J} sign conj(lam_row[J]) psi_row[I]
// over the listed excitations J = I - q + p; waves own (p, q) pairs and lanes
// take list entries, so every sum has a fixed order.  Tasks hold half the rows
// of a segment task (two states share the LDS rows).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rdm_rows_per_task(int seg_rows) { return seg_rows > 1 ? seg_rows / 2 : 1; }

template <class R, int CS>
__device__ __forceinline__ void rdm_task_cs(const BPassDev& ps, const BTypeDev& ty, int task, const BatchLds& L) {
  using V = typename V2T<R>::type;
  constexpr int cs = CS, rs = 1 - CS;
  const int N = ty.norb, NN = N * N;
  const int64_t nrows = pick2(ty.dim, rs), len = pick2(ty.dim, cs), ncols_state = ty.dim[1];
  const int RR = rdm_rows_per_task(pick2(ty.rows_per_task, cs));
  const int64_t r0 = (int64_t)task * RR;
  const int nr = (int)std::min<int64_t>(RR, nrows - r0);
  const int64_t nel = (int64_t)nr * len;
  const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  V* bl = (V*)L.rows;
  V* bp = bl + (int64_t)RR * len;
  const V* lam = (const V*)ps.src;
  const V* psi = (const V*)ps.src2;
  // staging: two elements of each state requested per thread before either is
  // stored (kept in named values: through arrays, the stores to LDS, which go
  // through a generic pointer, would keep the values in scratch memory); a task
  // holds at most 64 rows of at most 924 amplitudes, so indexes fit 32 bits
  const int ne = (int)nel;
  // the elements are copied as native two-component vectors (the same bytes)
  using T = typename std::conditional<sizeof(V) == 16, bdouble2, bfloat2>::type;
  T* tl = (T*)bl;
  T* tp = (T*)bp;
  if (ps.layout == 0) {
    const T* ls = (const T*)lam + r0 * len;
    const T* qs = (const T*)psi + r0 * len;
    for (int x0 = tid; x0 < ne; x0 += 2 * nthr) {
      const int x1 = min(x0 + nthr, ne - 1);
      const T a0 = ls[x0], b0 = qs[x0], a1 = ls[x1], b1 = qs[x1];
      tl[x0] = a0;
      tp[x0] = b0;
      tl[x1] = a1;
      tp[x1] = b1;
    }
  } else {
    const unsigned unr = (unsigned)nr, ulen = (unsigned)len;
    for (int x0 = tid; x0 < ne; x0 += 2 * nthr) {
      const unsigned y0 = (unsigned)x0, y1 = (unsigned)min(x0 + nthr, ne - 1);
      const unsigned k0 = y0 / unr, q0 = y0 - k0 * unr, k1 = y1 / unr, q1 = y1 - k1 * unr;
      const int64_t s0 = (int64_t)k0 * ncols_state + r0 + q0, s1 = (int64_t)k1 * ncols_state + r0 + q1;
      const T* tlam = (const T*)lam;
      const T* tpsi = (const T*)psi;
      const T a0 = tlam[s0], b0 = tpsi[s0], a1 = tlam[s1], b1 = tpsi[s1];
      tl[q0 * ulen + k0] = a0;
      tp[q0 * ulen + k0] = b0;
      tl[q1 * ulen + k1] = a1;
      tp[q1 * ulen + k1] = b1;
    }
  }
  __syncthreads();
  // T_pq = sum over rows and strings K of one electron fewer of
  // conj(lam[K + p]) psi[K + q] s_p(K) s_q(K), on the FP64 matrix cores: lane l
  // takes orbital l % 16 of string l / 16 of a block of four strings
  // (v_mfma_f64_16x16x4: A[l % 16][l / 16], B[l / 16][l % 16], result
  // D[l / 16 + 4 t][l % 16]); sums in a fixed order (per wave, then over waves)
  const int* kt = ty.kt[cs];
  const int nk = ty.nk[cs];
  const int o = lane & 15, kk = lane >> 4;
  bdouble4 rr = {0.0, 0.0, 0.0, 0.0}, ii = rr, ri = rr, ir = rr;
  const int nkb = (nk + 3) >> 2;
  for (int kb = wave; kb < nkb; kb += nw) {
    const int k = 4 * kb + kk;
    const int v = k < nk ? kt[k * 16 + o] : -1;
    const int64_t col = v >> 1;
    const bool neg = v & 1;
    for (int r = 0; r < nr; ++r) {
      double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
      if (v >= 0) {
        const V a = bl[(int64_t)r * len + col], b = bp[(int64_t)r * len + col];
        ar = (double)a.x;
        ai = (double)a.y;
        br = (double)b.x;
        bi = (double)b.y;
        if (neg) {
          ar = -ar;
          ai = -ai;
          br = -br;
          bi = -bi;
        }
      }
      rr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, rr, 0, 0, 0);
      ii = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, ii, 0, 0, 0);
      ri = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, ri, 0, 0, 0);
      ir = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, ir, 0, 0, 0);
    }
  }
  double* red = L.acc;  // [wave][re 256 | im 256]
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int pq = (kk + 4 * t) * 16 + o;
    red[wave * 512 + pq] = rr[t] + ii[t];
    red[wave * 512 + 256 + pq] = ri[t] - ir[t];
  }
  __syncthreads();
  for (int i = tid; i < NN; i += nthr) {
    const int p = i / N, q = i - p * N;
    double re = 0.0, im = 0.0;
    for (int w = 0; w < nw; ++w) {
      re += red[w * 512 + p * 16 + q];
      im += red[w * 512 + 256 + p * 16 + q];
    }
    ps.partials[(int64_t)task * 2 * NN + 2 * i] = re;
    ps.partials[(int64_t)task * 2 * NN + 2 * i + 1] = im;
  }
}

template <class R>
__device__ __forceinline__ void rdm_task(const BPassDev& ps, const BTypeDev& ty, int task, const BatchLds& L) {
  if (ps.layout == 0)
    rdm_task_cs<R, 1>(ps, ty, task, L);
  else
    rdm_task_cs<R, 0>(ps, ty, task, L);
}

// ---------------------------------------------------------------------------
// gradients of a LUCJ diagonal gate (same-spin pairs (p, p+1), opposite-spin
// pairs (p, p)), one wave per alpha row, with z = Im(conj(lam) psi):
//   out[p]       += 2 (x_a[p] x_a[p+1] sum z + sum z x_b[p] x_b[p+1])   p < N-1
//   out[N-1+p]   += 2 x_a[p] sum z x_b[p]
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void dgrad_task(const BPassDev& ps, const BTypeDev& ty, int task, double* acc) {
  using V = typename V2T<R>::type;
  const int N = ty.norb, NO = 2 * N - 1;
  const int64_t db = ty.dim[1];
  const int RR = ty.rows_per_task[1];
  const int64_t r0 = (int64_t)task * RR;
  const int nr = (int)std::min<int64_t>(RR, ty.dim[0] - r0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const V* lam = (const V*)ps.src;
  const V* psi = (const V*)ps.src2;
  double* out = acc + wave * 2 * kBatchMaxOrb;
  for (int i = threadIdx.x; i < 4 * 2 * kBatchMaxOrb; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  for (int r = wave; r < nr; r += nw) {
    const int64_t row = r0 + r;
    const uint32_t ma = ty.masks[0][row];
    double s0 = 0, s1[kBatchMaxOrb], s2[kBatchMaxOrb];
#pragma unroll
    for (int p = 0; p < kBatchMaxOrb; ++p) s1[p] = s2[p] = 0;
    for (int64_t k = lane; k < db; k += 64) {
      const V a = lam[row * db + k], b = psi[row * db + k];
      const double z = (double)a.x * (double)b.y - (double)a.y * (double)b.x;
      const uint32_t mb = ty.masks[1][k];
      s0 += z;
#pragma unroll
      for (int p = 0; p < kBatchMaxOrb; ++p) {
        const double bp = (double)((mb >> p) & 1);
        s1[p] += z * bp;
        s2[p] += z * bp * (double)((mb >> (p + 1)) & 1);
      }
    }
    s0 = wave_sum(s0);
#pragma unroll
    for (int p = 0; p < kBatchMaxOrb; ++p) {
      s1[p] = wave_sum(s1[p]);
      s2[p] = wave_sum(s2[p]);
    }
    if (lane == 0) {
#pragma unroll
      for (int p = 0; p < kBatchMaxOrb; ++p) {
        if (p + 1 < N) out[p] += 2.0 * ((double)(((ma >> p) & 1) & ((ma >> (p + 1)) & 1)) * s0 + s2[p]);
        if (p < N) out[N - 1 + p] += 2.0 * (double)((ma >> p) & 1) * s1[p];
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NO; i += blockDim.x) {
    double t = 0;
    for (int w = 0; w < nw; ++w) t += acc[w * 2 * kBatchMaxOrb + i];
    ps.partials[(int64_t)task * NO + i] = t;
  }
}

// ---------------------------------------------------------------------------
// segment pass on a block of rows (or columns) held back to back in LDS
// ---------------------------------------------------------------------------
template <int W, bool REAL, class R>
__device__ __forceinline__ void seg_task(const BatchDev& B, const BPassDev& ps, const BTypeDev& ty, int task, const BatchLds& L) {
  using V = typename V2T<R>::type;
  const int cs = ps.layout == 0 ? 1 : 0, rs = 1 - cs;
  const int N = ty.norb;
  const int64_t nrows = pick2(ty.dim, rs), len = pick2(ty.dim, cs), ncols_state = ty.dim[1];
  const int RR = pick2(ty.rows_per_task, cs);
  const void* src = ps.src;
  void* dst = ps.dst;
  if (task >= ps.half) {
    task -= ps.half;
    src = ps.src2;
    dst = ps.dst2;
  }
  const int64_t r0 = (int64_t)task * RR;
  const int nr = (int)std::min<int64_t>(RR, nrows - r0);
  const int64_t nel = (int64_t)nr * len;
  const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, nwaves = nthr >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave: chunk loops stay scalar
  V* buf = (V*)L.rows;
  const V* s = (const V*)src;

  // gather: element (r, k) of the layout lands at buf[r * len + k]; every
  // thread requests kU elements before it stores any.  A task holds at most
  // 64 rows of at most 924 amplitudes, so element indexes and their quotients
  // by the row count are taken in 32-bit unsigned arithmetic.
  constexpr int kU = 8;
  const int ne = (int)nel;
  const unsigned unr = (unsigned)nr, ulen = (unsigned)len;
  for (int x0 = tid; x0 < ne; x0 += kU * nthr) {
    V t[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const unsigned x = (unsigned)min(x0 + u * nthr, ne - 1);
      if (ps.layout == 0) {
        t[u] = s[r0 * len + x];
      } else {
        const unsigned k = x / unr, r = x - k * unr;
        t[u] = s[(int64_t)k * ncols_state + r0 + r];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) keep(t[u]);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int x = x0 + u * nthr;
      if (x < ne) {
        if (ps.layout == 0) {
          buf[x] = t[u];
        } else {
          const unsigned k = (unsigned)x / unr, r = (unsigned)x - k * unr;
          buf[r * ulen + k] = t[u];
        }
      }
    }
  }
  for (int64_t x = nel + tid; x < (int64_t)RR * len; x += nthr) buf[x] = V{};
  {
    // (the member-offset tables are a whole number of int4 words)
    const int n4 = pick2(ty.n_mt_all, cs) >> 2;
    const int4* m4 = (const int4*)pick2(ty.mt_all, cs);
    for (int i0 = tid; i0 < n4; i0 += 4 * nthr) {
      int4 q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = m4[min(i0 + u * nthr, n4 - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u) keep(q[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + u * nthr < n4) ((int4*)L.mt)[i0 + u * nthr] = q[u];
    }
  }
  __syncthreads();

  const uint32_t* cmask = pick2(ty.masks, cs);
  const uint32_t* rmask = pick2(ty.masks, rs) + r0;
  double acc = 0.0;
  // each Givens stage's rotations and first class codes are requested a stage
  // ahead (as in the segment pass)
  RotLane<R> rl_next{nullptr};
  ChunkAhead fc_next{1, 1, -1, -1};
  auto fetch = [&](int si) {
    const StageDev st = uniform_load(ps.stages + si);
    if (st.type == ST_GIVENS) {
      rl_next = fetch_rot_lane<R>(st.rots, st.nrot, lane);
      fc_next = fetch_first_chunk(uniform_load(pick2(ty.win, cs) + st.a), wave, lane, nwaves);
    }
  };
  if (ps.n_stages > 0) fetch(0);
  for (int si = 0; si < ps.n_stages; ++si) {
    const StageDev st = uniform_load(ps.stages + si);
    const RotLane<R> rl = rl_next;
    const ChunkAhead fc = fc_next;
    if (si + 1 < ps.n_stages) fetch(si + 1);
    if (st.type == ST_GIVENS) {
      const SegWinDev wt = uniform_load(pick2(ty.win, cs) + st.a);
      givens_stage<W, REAL, R>(st.shape, buf, L.mt, wt, rl, st.nrot, wave, nwaves, lane, fc);
    } else {
      // per row: cross weights w_r[q] = sum_{p in row} C[p][q] and the row factor
      for (int i = tid; i < nr * N; i += nthr) {
        const int r = i / N, q = i - r * N;
        double w = 0.0;
        if (st.C) {
          // the column of C is requested whole before the masked sum
          const uint32_t rm = rmask[r];
          double cq[kBatchMaxOrb];
#pragma unroll
          for (int p = 0; p < kBatchMaxOrb; ++p) cq[p] = st.C[min(p, N - 1) * N + q];
#pragma unroll
          for (int p = 0; p < kBatchMaxOrb; ++p)
            if (p < N && ((rm >> p) & 1)) w += cq[p];
        }
        L.wq[r * kBatchMaxOrb + q] = w;
      }
      for (int r = tid; r < nr; r += nthr) {
        const uint32_t rm = rmask[r];
        const double arow = st.A ? st.A[r0 + r] : 0.0;
        if (st.type == ST_PHASE) {
          double g = st.scale * arow;
          if (st.drow)
            for (uint32_t x = rm; x; x &= x - 1) g += st.drow[__builtin_ctz(x)];
          zc128 f = phase_factor<double>(g);
          if (__builtin_popcount(rm & st.sign_row) & 1) {
            f.x = -f.x;
            f.y = -f.y;
          }
          L.rowf[2 * r] = f.x;
          L.rowf[2 * r + 1] = f.y;
        } else {
          L.rowf[2 * r] = arow;
        }
      }
      __syncthreads();
      const bool cross = st.C != nullptr;
      for (int x = tid; x < ne; x += nthr) {
        const unsigned r = (unsigned)x / ulen, k = (unsigned)x - r * ulen;
        double cr = 0.0;
        if (cross)
          for (uint32_t b = cmask[k]; b; b &= b - 1) cr += L.wq[r * kBatchMaxOrb + __builtin_ctz(b)];
        V y = buf[x];
        if (st.type == ST_PHASE) {
          zc128 f{L.rowf[2 * r], L.rowf[2 * r + 1]};
          if (st.colf) f = zmul(f, ((const zc128*)st.colf)[k]);
          if (__builtin_popcount(cmask[k] & st.sign_col) & 1) {
            f.x = -f.x;
            f.y = -f.y;
          }
          if (cross) {
            const V e = phase_factor<R>(st.scale * cr);
            f = zmul(f, zc128{(double)e.x, (double)e.y});
          }
          V o;
          o.x = (R)((double)y.x * f.x - (double)y.y * f.y);
          o.y = (R)((double)y.x * f.y + (double)y.y * f.x);
          buf[x] = o;
        } else {
          const double f = L.rowf[2 * r] + (st.B ? st.B[k] : 0.0) + cr;
          if (st.type == ST_SCALE) {
            y.x = (R)(f * (double)y.x);
            y.y = (R)(f * (double)y.y);
            buf[x] = y;
          } else {
            acc += f * ((double)y.x * (double)y.x + (double)y.y * (double)y.y);
          }
        }
      }
    }
    __syncthreads();
  }

  if (ps.mode != SEG_NONE) {
    V* d = (V*)dst;
    const bool add = ps.mode == SEG_ACCUM;
    if (ps.layout == 0) {
      for (int x = tid; x < ne; x += nthr) {
        V v = buf[x];
        if (add) {
          const V a = d[r0 * len + x];
          v.x += a.x;
          v.y += a.y;
        }
        d[r0 * len + x] = v;
      }
    } else {
      for (int x = tid; x < ne; x += nthr) {
        const unsigned k = (unsigned)x / unr, r = (unsigned)x - k * unr;
        const int64_t gi = (int64_t)k * ncols_state + r0 + r;
        V v = buf[r * ulen + k];
        if (add) {
          const V a = d[gi];
          v.x += a.x;
          v.y += a.y;
        }
        d[gi] = v;
      }
    }
  }
  if (ps.partials) {
    const double t = batch_block_sum(acc, L.red);
    if (tid == 0) ps.partials[task] = t;
  }
}

// ---------------------------------------------------------------------------
// the persistent kernel
// ---------------------------------------------------------------------------
template <int W, class R>
__global__ __launch_bounds__(kBatchThreads) void k_batch(BatchDev B) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_pass, s_ok;
  __shared__ int64_t s_task;
  const BatchLds L = batch_lds_map(smem, B);
  for (;;) {
    if (threadIdx.x == 0) {
      int pi = -1;
      int64_t t = -1;
      if (!__hip_atomic_load(B.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        t = (int64_t)__hip_atomic_fetch_add(B.next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t < B.n_tasks) {
          int lo = 0, hi = B.n_passes - 1;  // last pass whose first task <= t
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (B.passes[mid].first <= t)
              lo = mid;
            else
              hi = mid - 1;
          }
          pi = lo;
        }
      }
      int ok = pi >= 0;
      if (ok) {
        const int inst = B.passes[pi].inst;
        const unsigned need = (unsigned)B.passes[pi].need;
        // poll with relaxed loads (an acquire here would invalidate the caches on
        // every iteration under the other blocks' running tasks); the acquire
        // fence after the barrier below orders this block's reads of the data
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        while (__hip_atomic_load(B.done + inst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(32);
          if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks ||
              __hip_atomic_load(B.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(B.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
        }
      }
      s_pass = pi;
      s_task = t;
      s_ok = ok;
    }
    __syncthreads();
    const int pi = s_pass;
    const int64_t t = s_task;
    const int ok = s_ok;
    __syncthreads();
    if (!ok) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const BPassDev ps = uniform_load(B.passes + pi);
    const BTypeDev ty = uniform_load(B.types + ps.type);
    const int task = (int)(t - ps.first);
    switch (ps.kind) {
      case BK_TABLES: tables_task(ps, ty, task); break;
      case BK_OUTER: outer_task<R>(ps, ty, task); break;
      case BK_SEG:
        if (ps.real)
          seg_task<W, true, R>(B, ps, ty, task, L);
        else
          seg_task<W, false, R>(B, ps, ty, task, L);
        break;
      case BK_INNER: inner_task<R>(ps, ty, task, L.red); break;
      case BK_RDM: rdm_task<R>(ps, ty, task, L); break;
      case BK_DGRAD: dgrad_task<R>(ps, ty, task, L.acc); break;
      case BK_SUM: sum_task(ps); break;
      default: break;
    }
    // publish this task's writes device-wide, then count it as finished
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(B.done + ps.inst, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Level-synchronous form: one launch runs the passes [p0, p1) of one level
// that all have kind KIND (the host groups a level's passes by kind), one block
// per task; ordering between levels comes from the launches.  Each launch
// carries only its kind's code, so its register count, and with it the number
// of blocks a compute unit holds, is that kind's own rather than the largest of
// all (segment tasks: 126 registers for complex64 instead of 196).
template <int W, class R, int KIND>
__global__ __launch_bounds__(kBatchThreads) void k_batch_kind(BatchDev B, int p0, int p1) {
  extern __shared__ __align__(16) char smem[];
  const BatchLds L = batch_lds_map(smem, B, KIND);
  const int64_t t = B.passes[p0].first + (int64_t)blockIdx.x;
  int lo = p0, hi = p1 - 1;  // last pass of the group whose first task <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (B.passes[mid].first <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const BPassDev ps = uniform_load(B.passes + lo);
  const BTypeDev ty = uniform_load(B.types + ps.type);
  const int task = (int)(t - ps.first);
  if (task < 0 || task >= ps.n_tasks) return;
  if constexpr (KIND == BK_TABLES) tables_task(ps, ty, task);
  if constexpr (KIND == BK_OUTER) outer_task<R>(ps, ty, task);
  if constexpr (KIND == BK_SEG) {
    if (ps.real)
      seg_task<W, true, R>(B, ps, ty, task, L);
    else
      seg_task<W, false, R>(B, ps, ty, task, L);
  }
  if constexpr (KIND == BK_INNER) inner_task<R>(ps, ty, task, L.red);
  if constexpr (KIND == BK_RDM) rdm_task<R>(ps, ty, task, L);
  if constexpr (KIND == BK_DGRAD) dgrad_task<R>(ps, ty, task, L.acc);
  if constexpr (KIND == BK_SUM) sum_task(ps);
}

// Single cooperative launch: every block walks the levels in order, taking
// the tasks of the current level from a per-level counter (zeroed before the
// launch; a block only ever increments it, and leaves the level once it runs
// past the level's last task), and the whole grid meets at a grid barrier
// between levels (the same ordering the per-level launches get from the
// launch boundaries).  Every block reaches every barrier.
template <int W, class R>
__global__ __launch_bounds__(kBatchThreads) void k_batch_coop(BatchDev B, const int* __restrict__ level_start,
                                                              int n_levels, unsigned int* __restrict__ level_ctr) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int64_t s_t;
  const BatchLds L = batch_lds_map(smem, B);
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int lv = 0; lv < n_levels; ++lv) {
    const int p0 = level_start[lv], p1 = level_start[lv + 1];
    if (p0 < p1) {
      const int64_t t0 = B.passes[p0].first;
      const int64_t t1 = p1 < B.n_passes ? B.passes[p1].first : B.n_tasks;
      for (;;) {
        if (threadIdx.x == 0) s_t = t0 + (int64_t)atomicAdd(level_ctr + lv, 1u);
        __syncthreads();
        const int64_t t = s_t;
        __syncthreads();
        if (t >= t1) break;
        int lo = p0, hi = p1 - 1;  // last pass of the level whose first task <= t
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (B.passes[mid].first <= t)
            lo = mid;
          else
            hi = mid - 1;
        }
        const BPassDev ps = uniform_load(B.passes + lo);
        const BTypeDev ty = uniform_load(B.types + ps.type);
        const int task = (int)(t - ps.first);
        if (task >= 0 && task < ps.n_tasks) {
          switch (ps.kind) {
            case BK_TABLES: tables_task(ps, ty, task); break;
            case BK_OUTER: outer_task<R>(ps, ty, task); break;
            case BK_SEG:
              if (ps.real)
                seg_task<W, true, R>(B, ps, ty, task, L);
              else
                seg_task<W, false, R>(B, ps, ty, task, L);
              break;
            case BK_INNER: inner_task<R>(ps, ty, task, L.red); break;
            case BK_RDM: rdm_task<R>(ps, ty, task, L); break;
            case BK_DGRAD: dgrad_task<R>(ps, ty, task, L.acc); break;
            case BK_SUM: sum_task(ps); break;
            default: break;
          }
        }
        __syncthreads();  // the next task of this block reuses the LDS
      }
    }
    grid.sync();
  }
}

template <int W, class R>
static hipError_t launch_coop(const BatchDev& b, const int* level_start, int n_levels, unsigned int* level_ctr,
                              int blocks, size_t lds, hipStream_t s) {
  auto k = k_batch_coop<W, R>;
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, kBatchMaxDynLds);
  (void)hipGetLastError();
  BatchDev bb = b;
  const int* ls = level_start;
  int nl = n_levels;
  unsigned int* lc = level_ctr;
  void* args[] = {(void*)&bb, (void*)&ls, (void*)&nl, (void*)&lc};
  return hipLaunchCooperativeKernel((const void*)k, dim3((unsigned)blocks), dim3(kBatchThreads), args,
                                    (unsigned)lds, s);
}

int batch_coop_blocks_per_cu(bool c64, size_t lds) {
  int n = 0;
  hipError_t e;
  if (lds > (size_t)kBatchMaxDynLds) return 0;
  if (c64) {
    (void)hipFuncSetAttribute((const void*)k_batch_coop<6, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kBatchMaxDynLds);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_coop<6, float>, kBatchThreads, lds);
  } else {
    (void)hipFuncSetAttribute((const void*)k_batch_coop<6, double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kBatchMaxDynLds);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_coop<6, double>, kBatchThreads, lds);
  }
  (void)hipGetLastError();
  return e == hipSuccess ? n : 0;
}

hipError_t batch_launch_coop(bool c64, const BatchDev& b, const int* level_start, int n_levels,
                             unsigned int* level_ctr, int blocks, size_t lds, hipStream_t s) {
  return c64 ? launch_coop<6, float>(b, level_start, n_levels, level_ctr, blocks, lds, s)
             : launch_coop<6, double>(b, level_start, n_levels, level_ctr, blocks, lds, s);
}

template <int W, class R, int KIND>
static void launch_kind(const BatchDev& b, int p0, int p1, int64_t tasks, size_t lds, hipStream_t s) {
  auto k = k_batch_kind<W, R, KIND>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, kBatchMaxDynLds);
    (void)hipGetLastError();
    attr_set = true;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)tasks), dim3(kBatchThreads), lds, s, b, p0, p1);
}

template <class R>
static void launch_kind_r(int kind, const BatchDev& b, int p0, int p1, int64_t tasks, size_t lds, hipStream_t s) {
  switch (kind) {
    case BK_TABLES: launch_kind<6, R, BK_TABLES>(b, p0, p1, tasks, lds, s); break;
    case BK_OUTER: launch_kind<6, R, BK_OUTER>(b, p0, p1, tasks, lds, s); break;
    case BK_SEG: launch_kind<6, R, BK_SEG>(b, p0, p1, tasks, lds, s); break;
    case BK_INNER: launch_kind<6, R, BK_INNER>(b, p0, p1, tasks, lds, s); break;
    case BK_RDM: launch_kind<6, R, BK_RDM>(b, p0, p1, tasks, lds, s); break;
    case BK_DGRAD: launch_kind<6, R, BK_DGRAD>(b, p0, p1, tasks, lds, s); break;
    case BK_SUM: launch_kind<6, R, BK_SUM>(b, p0, p1, tasks, lds, s); break;
    default: break;
  }
}

void batch_launch_kind(bool c64, int kind, const BatchDev& b, int p0, int p1, int64_t tasks, size_t lds,
                       hipStream_t s) {
  if (c64)
    launch_kind_r<float>(kind, b, p0, p1, tasks, lds, s);
  else
    launch_kind_r<double>(kind, b, p0, p1, tasks, lds, s);
}


template <int W, class R>
static void launch_batch(const BatchDev& b, int blocks, int threads, size_t lds, hipStream_t s) {
  auto k = k_batch<W, R>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, kBatchMaxDynLds);
    (void)hipGetLastError();
    attr_set = true;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(threads), lds, s, b);
}

int batch_blocks_per_cu(bool c64, int threads, size_t lds) {
  int n = 0;
  hipError_t e;
  if (lds > (size_t)kBatchMaxDynLds) return 0;
  if (c64) {
    (void)hipFuncSetAttribute((const void*)k_batch<6, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kBatchMaxDynLds);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<6, float>, threads, lds);
  } else {
    (void)hipFuncSetAttribute((const void*)k_batch<6, double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kBatchMaxDynLds);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<6, double>, threads, lds);
  }
  (void)hipGetLastError();
  return e == hipSuccess ? n : 0;
}

void batch_launch(bool c64, const BatchDev& b, int blocks, int threads, size_t lds, hipStream_t s) {
  if (c64)
    launch_batch<6, float>(b, blocks, threads, lds, s);
  else
    launch_batch<6, double>(b, blocks, threads, lds, s);
}

}  // namespace dev
}  // namespace ffx
