// Sampling of configurations (Sec. 4.5.4 and 6.1):
//   * from a state vector, by the inverse of its cumulative distribution
//     |gamma|^2 in address order (FP64, fixed summation order);
//   * from a Slater determinant without forming the state: per spin, the
//     projection determinantal point process with kernel K = Q Q^dag
//     (Q = the occupied columns of the orbital rotation), drawn one orbital
//     at a time from its conditional distribution (O(eta^2 N) per sample).
// Uniform random numbers come in from the caller.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "dev_common.h"
#include "device.h"

namespace ffx {
namespace dev {

constexpr int64_t kNone = 0x7fffffffffffffffLL;
constexpr int kSampleChunk = 4;                   // amplitudes per thread
constexpr int kSampleBlock = 256 * kSampleChunk;  // amplitudes per block (16 KB of complex128 read per sample)

int sample_blocks(int64_t n) { return (int)((n + kSampleBlock - 1) / kSampleBlock); }

constexpr int64_t kSearchChunk = (int64_t)1 << 24;  // samples per search launch

// bs[b] = sum |gamma|^2 over block b (kSampleBlock addresses from b *
// kSampleBlock): thread t sums addresses t, t + 256, t + 2 * 256, ... of the
// block in that order (so that each load instruction of a wave reads
// consecutive amplitudes), then the fixed tree of block_sum256
template <class R>
__global__ __launch_bounds__(256) void k_block_norm2(const typename V2T<R>::type* __restrict__ v, int64_t n,
                                                     double* __restrict__ bs) {
  using V = typename V2T<R>::type;
  __shared__ double sh[4];
  const int64_t base = (int64_t)blockIdx.x * kSampleBlock + threadIdx.x;
  V x[kSampleChunk];
#pragma unroll
  for (int k = 0; k < kSampleChunk; ++k) {
    const int64_t i = base + (int64_t)k * 256;
    x[k] = i < n ? v[i] : V{R(0), R(0)};
  }
  double acc = 0;
#pragma unroll
  for (int k = 0; k < kSampleChunk; ++k) {
    const double re = x[k].x, im = x[k].y;
    acc += re * re + im * im;
  }
  const double t = block_sum256(acc, sh);
  if (threadIdx.x == 0) bs[blockIdx.x] = t;
}

// inclusive prefix of bs[0..nb) into pre, one block of 1024 threads: each
// thread scans a contiguous chunk, thread 0 scans the chunk totals in order.
// A thread's loads are requested 16 at a time (indexes clamped into its chunk,
// so no load waits behind a branch) before the sequential additions use them.
__global__ __launch_bounds__(1024) void k_scan_blocks(const double* __restrict__ bs, int nb,
                                                      double* __restrict__ pre) {
  __shared__ double tot[1024];
  constexpr int B = 16;
  const int c = (nb + 1023) / 1024;
  const int lo = min((int)threadIdx.x * c, nb), hi = min(nb, lo + c);
  double run = 0;
  for (int i0 = lo; i0 < hi; i0 += B) {
    double x[B];
#pragma unroll
    for (int k = 0; k < B; ++k) x[k] = bs[min(i0 + k, hi - 1)];
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (i0 + k < hi) {
        run += x[k];
        pre[i0 + k] = run;
      }
  }
  tot[threadIdx.x] = run;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0;
    for (int t = 0; t < 1024; ++t) {
      const double x = tot[t];
      tot[t] = acc;
      acc += x;
    }
  }
  __syncthreads();
  const double off = tot[threadIdx.x];
  for (int i0 = lo; i0 < hi; i0 += B) {
    double x[B];
#pragma unroll
    for (int k = 0; k < B; ++k) x[k] = pre[min(i0 + k, hi - 1)];
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (i0 + k < hi) pre[i0 + k] = x[k] + off;
  }
}

// One block per sample: the first address whose cumulative probability exceeds
// u * total (zero-probability addresses are never chosen; when rounding leaves
// the target at or past the block's own total, the block's last address with
// nonzero probability).
//   * Block search: the first b with pre[b] > target (else nb - 1), by rounds
//     in which the 256 threads test 256 evenly spaced entries of the remaining
//     range at once (pre never decreases, so the entries that fail form a
//     prefix; their count narrows the range 256-fold per round).
//   * In-block search: thread t sums its kSampleChunk consecutive amplitudes; the
//     exclusive prefix of those sums in thread order comes from a shuffle scan
//     within each wave plus the totals of the waves before it (a fixed order);
//     then each thread walks its own amplitudes.
template <class R>
__global__ __launch_bounds__(256) void k_sample_search(const typename V2T<R>::type* __restrict__ v, int64_t n,
                                                       const double* __restrict__ pre, int nb,
                                                       const double* __restrict__ u, int64_t n_samples,
                                                       int64_t* __restrict__ out) {
  __shared__ double wtot[4];
  __shared__ int64_t sel[2];
  const int64_t s = blockIdx.x;
  if (s >= n_samples) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double total = pre[nb - 1];
  const double us = u[s];
  // (the same decision in every thread of the block) a state without a finite
  // nonzero norm, or a uniform outside [0, 1), gives -1
  if (!(total > 0.0) || !isfinite(total) || !(us >= 0.0 && us < 1.0)) {
    if (tid == 0) out[s] = -1;
    return;
  }
  const double target = us * total;
  if (tid == 0) {
    sel[0] = kNone;  // first qualifying address
    sel[1] = -1;     // last address with nonzero probability
  }
  int lo = 0, hi = nb - 1;  // the answer lies in [lo, hi]
  while (lo < hi) {
    const int step = (hi - lo + 256) / 256;  // ceil((hi - lo + 1) / 256)
    const int i = min(lo + (tid + 1) * step - 1, hi);
    const int c = __syncthreads_count(!(pre[i] > target));  // entries tested that fail
    if (c == 256) {
      lo = hi;  // every tested entry fails, hi among them: the answer is hi
    } else {
      const int nlo = c == 0 ? lo : min(lo + c * step - 1, hi) + 1;
      hi = min(lo + (c + 1) * step - 1, hi);
      lo = nlo;
    }
  }
  const int b = lo;
  const double t2 = target - (b > 0 ? pre[b - 1] : 0.0);
  const int64_t base = (int64_t)b * kSampleBlock + (int64_t)tid * kSampleChunk;
  double w[kSampleChunk];
  double acc = 0;
#pragma unroll
  for (int k = 0; k < kSampleChunk; ++k) {
    const int64_t i = base + k;
    double p = 0;
    if (i < n) {
      const double re = v[i].x, im = v[i].y;
      p = re * re + im * im;
    }
    w[k] = p;
    acc += p;
  }
  // inclusive scan of the thread sums within the wave
  double inc = acc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wtot[wave] = inc;
  const double excl = __shfl_up(inc, 1);
  __syncthreads();
  double cum = 0;
  for (int q = 0; q < wave; ++q) cum += wtot[q];
  if (lane > 0) cum += excl;
  int64_t first = kNone, last = -1;
#pragma unroll
  for (int k = 0; k < kSampleChunk; ++k) {
    if (w[k] > 0) {
      cum += w[k];
      last = base + k;
      if (first == kNone && cum > t2) first = base + k;
    }
  }
  if (first != kNone) atomicMin((unsigned long long*)&sel[0], (unsigned long long)first);
  if (last >= 0) atomicMax((long long*)&sel[1], (long long)last);
  __syncthreads();
  if (tid == 0) out[s] = sel[0] != kNone ? sel[0] : sel[1];
}

int sample_state(bool c64, const void* vec, int64_t n, double* bs, double* pre, const double* u, int64_t n_samples,
                 int64_t* out, hipStream_t s) {
  const int nb = sample_blocks(n);
  if (c64) {
    hipLaunchKernelGGL(k_block_norm2<float>, dim3(nb), dim3(256), 0, s, (const zc64*)vec, n, bs);
  } else {
    hipLaunchKernelGGL(k_block_norm2<double>, dim3(nb), dim3(256), 0, s, (const zc128*)vec, n, bs);
  }
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, bs, nb, pre);
  // one block per sample, at most kSearchChunk blocks per launch (the grid's
  // work-items stay below 2^32)
  for (int64_t off = 0; off < n_samples; off += kSearchChunk) {
    const int64_t cnt = n_samples - off < kSearchChunk ? n_samples - off : kSearchChunk;
    const dim3 g((unsigned)cnt);
    if (c64)
      hipLaunchKernelGGL(k_sample_search<float>, g, dim3(256), 0, s, (const zc64*)vec, n, pre, nb, u + off, cnt,
                         out + off);
    else
      hipLaunchKernelGGL(k_sample_search<double>, g, dim3(256), 0, s, (const zc128*)vec, n, pre, nb, u + off, cnt,
                         out + off);
  }
  return nb;
}

// Device memory of the allocation-free state sampler: the block sums and
// their prefix, 2 * kScratchBlocks doubles (4 MiB) per device, held until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device array: its device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address is used.
__device__ __align__(256) double scratch[2 * kScratchBlocks];

hipError_t sample_scratch(int device, double** ptr) {
  static std::mutex mu;
  static std::vector<double*> addr;
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = (double*)p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Slater determinant: one wavefront per sample and spin.  Lane j < N holds the
// residual weight r_j = |q_j|^2 - sum_i |<e_i, q_j>|^2 of row j of Q (N x eta,
// complex, in LDS) against the orthonormal basis e_0.. of the rows chosen so
// far (kept in LDS per wave).  Step k: lane 0 picks the first j whose
// cumulative r (in orbital order) exceeds u_k * sum r; the new basis vector is
// the chosen row minus its projections, normalised; every lane then removes
// its overlap with it.
// LDS (dynamic, sized by N and eta): Q (N x eta), then per wave the basis
// (eta x eta) and the overlaps <e_i, q_j> (N x eta, at [j][i]); up to
// kDppWaves waves per block, fewer where the arrays would pass 64 KB.
// ---------------------------------------------------------------------------
constexpr int kDppWaves = 4;
constexpr size_t kDppLdsCap = 64 * 1024;

static size_t dpp_wave_doubles(int N, int eta) { return (size_t)2 * eta * eta + (size_t)2 * N * eta; }

__global__ __launch_bounds__(64 * kDppWaves) void k_dpp_sample(const double* __restrict__ Q, int N, int eta,
                                                                 const double* __restrict__ u, int64_t n_samples,
                                                                 uint64_t* __restrict__ masks) {
  extern __shared__ double dsm[];
  __shared__ double rr[kDppWaves][32];
  __shared__ int pick[kDppWaves];
  const int nq = N * eta * 2;
  double* q = dsm;
  for (int i = threadIdx.x; i < nq; i += blockDim.x) q[i] = Q[i];
  __syncthreads();
  const int waves = blockDim.x >> 6;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* e = dsm + nq + (size_t)wv * (2 * eta * eta + nq);  // e_i component c at [i][c]
  double* coef = e + 2 * eta * eta;                            // <e_i, q_j> at [j][i]
  const int64_t smp = (int64_t)blockIdx.x * waves + wv;
  if (smp >= n_samples) return;  // whole waves leave together; no block barrier follows
  double r = 0;
  if (lane < N)
    for (int c = 0; c < eta; ++c) {
      const double a = q[(lane * eta + c) * 2], bi = q[(lane * eta + c) * 2 + 1];
      r += a * a + bi * bi;
    }
  uint64_t mask = 0;
  for (int k = 0; k < eta; ++k) {
    if (lane < N) rr[wv][lane] = ((mask >> lane) & 1) ? 0.0 : (r > 0 ? r : 0.0);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (lane == 0) {
      double tot = 0;
      for (int j = 0; j < N; ++j) tot += rr[wv][j];
      const double target = u[smp * eta + k] * tot;
      double cum = 0;
      int first = -1, last = -1;
      for (int j = 0; j < N; ++j) {
        const double x = rr[wv][j];
        if (x > 0) {
          cum += x;
          last = j;
          if (first < 0 && cum > target) first = j;
        }
      }
      pick[wv] = first >= 0 ? first : last;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const int js = pick[wv];
    if (js < 0) break;  // no weight left (cannot happen for orthonormal columns)
    mask |= 1ull << js;
    // e_k = (q_js - sum_{i<k} <e_i, q_js> e_i) / |...|, component c on lane c
    const double rjs = rr[wv][js];
    const double inv = 1.0 / sqrt(rjs);
    if (lane < eta) {
      double vr = q[(js * eta + lane) * 2], vi = q[(js * eta + lane) * 2 + 1];
      for (int i = 0; i < k; ++i) {
        const double cr = coef[(js * eta + i) * 2], ci = coef[(js * eta + i) * 2 + 1];
        const double er = e[(i * eta + lane) * 2], ei = e[(i * eta + lane) * 2 + 1];
        vr -= cr * er - ci * ei;
        vi -= cr * ei + ci * er;
      }
      e[(k * eta + lane) * 2] = vr * inv;
      e[(k * eta + lane) * 2 + 1] = vi * inv;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (lane < N) {
      double cr = 0, ci = 0;  // <e_k, q_lane> = sum conj(e) q
      for (int c = 0; c < eta; ++c) {
        const double er = e[(k * eta + c) * 2], ei = e[(k * eta + c) * 2 + 1];
        const double a = q[(lane * eta + c) * 2], bi = q[(lane * eta + c) * 2 + 1];
        cr += er * a + ei * bi;
        ci += er * bi - ei * a;
      }
      coef[(lane * eta + k) * 2] = cr;
      coef[(lane * eta + k) * 2 + 1] = ci;
      r -= cr * cr + ci * ci;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  }
  if (lane == 0) masks[smp] = mask;
}

void dpp_sample(const double* Q, int N, int eta, const double* u, int64_t n_samples, uint64_t* masks,
                hipStream_t s) {
  if (n_samples <= 0) return;
  const size_t qd = (size_t)2 * N * eta, wd = dpp_wave_doubles(N, eta);
  int waves = kDppWaves;
  while (waves > 1 && (qd + waves * wd) * sizeof(double) > kDppLdsCap) --waves;
  const size_t lds = (qd + waves * wd) * sizeof(double);  // at most 48 KB at N = eta = 32
  // at most kSearchChunk samples per launch (the grid's work-items stay below 2^32)
  for (int64_t off = 0; off < n_samples; off += kSearchChunk) {
    const int64_t cnt = n_samples - off < kSearchChunk ? n_samples - off : kSearchChunk;
    const dim3 g((unsigned)((cnt + waves - 1) / waves));
    hipLaunchKernelGGL(k_dpp_sample, g, dim3(64 * waves), lds, s, Q, N, eta, u + off * eta, cnt, masks + off);
  }
}

}  // namespace dev
}  // namespace ffx
