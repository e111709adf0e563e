// Device-side helpers shared by the HIP translation units of libffx:
// complex amplitude types, compile-time pattern / pair tables of a window, the
// register-resident Givens application, phase factors and block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>
#include <utility>

#include "device.h"

namespace ffx {
namespace dev {

// Complex amplitudes as plain aligned structs (HIP's union-based vector types
// keep register arrays of them from being promoted out of scratch memory).
struct alignas(16) zc128 {
  double x, y;
};
struct alignas(8) zc64 {
  float x, y;
};
template <class R>
struct V2T;
template <>
struct V2T<double> {
  using type = zc128;
};
template <>
struct V2T<float> {
  using type = zc64;
};

// One part (real or imaginary) of a complex128 amplitude: the element of a
// row plane, which real Givens rotations act on independently of the other.
struct re128 {
  double x;
};

// The scalar type of an element type, and whether the element is a single
// plane part (real rotations only).
template <class V>
struct ElemT;
template <>
struct ElemT<zc128> {
  using R = double;
  static constexpr bool plane = false;
};
template <>
struct ElemT<zc64> {
  using R = float;
  static constexpr bool plane = false;
};
template <>
struct ElemT<re128> {
  using R = double;
  static constexpr bool plane = true;
};
template <class V>
using ER = typename ElemT<V>::R;

constexpr int cbinom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long long r = 1;
  for (int i = 0; i < k; ++i) r = r * (n - i) / (i + 1);
  return (int)r;
}

struct BinomTab {
  int v[33][33];
  constexpr BinomTab() : v{} {
    for (int n = 0; n <= 32; ++n)
      for (int k = 0; k <= 32; ++k) v[n][k] = cbinom(n, k);
  }
};
static __constant__ const BinomTab kBinom = BinomTab();

// address of a configuration: sum_k C(i_k, k) over its set bits i_1 < i_2 < ...
__device__ __forceinline__ int colex_rank(uint32_t m) {
  int r = 0, k = 1;
  while (m) {
    int i = __builtin_ctz(m);
    r += kBinom.v[i][k++];
    m &= m - 1;
  }
  return r;
}

// ---------------------------------------------------------------------------
// compile-time pattern and pair tables
// ---------------------------------------------------------------------------
template <int W, int M>
struct Pat {
  static constexpr int C = cbinom(W, M);
  int mask[C > 0 ? C : 1];
  constexpr Pat() : mask{} {
    int k = 0;
    for (int x = 0; x < (1 << W); ++x) {
      int pc = 0;
      for (int b = 0; b < W; ++b) pc += (x >> b) & 1;
      if (pc == M) mask[k++] = x;
    }
  }
  constexpr int index(int x) const {
    for (int k = 0; k < C; ++k)
      if (mask[k] == x) return k;
    return -1;
  }
};

template <int W, int M, int P>
struct Pairs {
  static constexpr int NP = cbinom(W - 2, M - 1);
  int a[NP > 0 ? NP : 1];
  int b[NP > 0 ? NP : 1];
  constexpr Pairs() : a{}, b{} {
    Pat<W, M> pt{};
    int n = 0;
    for (int k = 0; k < Pat<W, M>::C; ++k) {
      int x = pt.mask[k];
      if (((x >> P) & 1) && !((x >> (P + 1)) & 1)) {
        a[n] = k;
        b[n] = pt.index(x ^ (3 << P));
        ++n;
      }
    }
  }
};

template <class V, class R>
__device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// d <- a * d + b and d <- a * b + d, written into d's own register: with the
// result tied to the input, the member registers never move across the
// rotation loop.  a is a rotation parameter, the same in every lane: it is
// read from scalar registers (one scalar operand per instruction, within the
// constant-bus limit), so it needs no copy into vector registers.
__device__ __forceinline__ void fma_ip(float& d, float a, float b) {
  asm("v_fma_f32 %0, %1, %0, %2" : "+v"(d) : "s"(a), "v"(b));
}
__device__ __forceinline__ void fma_ip(double& d, double a, double b) {
  asm("v_fma_f64 %0, %1, %0, %2" : "+v"(d) : "s"(a), "v"(b));
}
__device__ __forceinline__ void fma_acc(float& d, float a, float b) {
  asm("v_fma_f32 %0, %1, %2, %0" : "+v"(d) : "s"(a), "v"(b));
}
__device__ __forceinline__ void fma_acc(double& d, double a, double b) {
  asm("v_fma_f64 %0, %1, %2, %0" : "+v"(d) : "s"(a), "v"(b));
}

// The parameters of one rotation as the rotation code takes them.  Complex
// sine: (c, sr, si).  Real sine: the rotation [[c, s], [-s, c]] with c >= 0
// (every cosine of a decomposition is) is the product of three shears,
// [[1, t], [0, 1]] [[1, 0], [b, 1]] [[1, t], [0, 1]] with t = s / (1 + c) and
// b = -s (1 + t b = c and t (1 + c) = s), so each component of a member pair
// takes three in-place FMAs, x += t y, y += b x, x += t y, instead of two
// multiplications and two FMAs; |t| <= 1, so the shears add no more than
// ordinary rounding.
template <class R>
struct RotShear {
  R t, b;
};
template <class R>
struct RotCplx {
  R c, sr, si;
};
template <bool REAL, class R>
using RotQ = typename std::conditional<REAL, RotShear<R>, RotCplx<R>>::type;

// one component of a member pair under the three shears
template <class R>
__device__ __forceinline__ void shear3(R& x, R& y, R t, R b) {
  fma_acc(x, t, y);
  fma_acc(y, b, x);
  fma_acc(x, t, y);
}

// x' = c x + s y, y' = -conj(s) x + c y on one member pair (A, B)
template <int A, int B, bool REAL, class V>
__device__ __forceinline__ void rot_pair(V* v, const RotQ<REAL, ER<V>>& q) {
  using R = ER<V>;
  V& x = v[A];
  V& y = v[B];
  if constexpr (ElemT<V>::plane) {
    // one plane of the row: a real rotation acts on it alone
    static_assert(REAL, "row planes take real rotations only");
    shear3<R>(x.x, y.x, q.t, q.b);
  } else if constexpr (REAL) {
    shear3<R>(x.x, y.x, q.t, q.b);
    shear3<R>(x.y, y.y, q.t, q.b);
  } else {
    const R c = q.c, sr = q.sr, si = q.si;
    const R tx = sr * y.x - si * y.y;
    const R ty = sr * y.y + si * y.x;
    const R ux = -sr * x.x - si * x.y;
    const R uy = si * x.x - sr * x.y;
    fma_ip(x.x, c, tx);
    fma_ip(x.y, c, ty);
    fma_ip(y.x, c, ux);
    fma_ip(y.y, c, uy);
  }
}

// every member pair of rotation P, expanded at compile time so that the
// register array is only ever indexed by constants
template <int W, int M, int P, bool REAL, class V, int... I>
__device__ __forceinline__ void rot_pairs(V* v, const RotQ<REAL, ER<V>>& q, std::integer_sequence<int, I...>) {
  constexpr Pairs<W, M, P> pr{};
  (rot_pair<pr.a[I], pr.b[I], REAL, V>(v, q), ...);
}

template <int W, int M, int P, bool REAL, class V>
__device__ __forceinline__ void rot_one(V* v, const RotQ<REAL, ER<V>>& q) {
  rot_pairs<W, M, P, REAL, V>(v, q, std::make_integer_sequence<int, Pairs<W, M, P>::NP>{});
}

template <int W, int M, bool REAL, class V, int P = 0>
__device__ __forceinline__ void rot_dispatch(int p, V* v, const RotQ<REAL, ER<V>>& q) {
  if constexpr (P < W - 1) {
    if (p == P)
      rot_one<W, M, P, REAL, V>(v, q);
    else
      rot_dispatch<W, M, REAL, V, P + 1>(p, v, q);
  }
}

// the rotation code's parameters from a RotDev, in the element's precision
template <bool REAL, class R>
__device__ __forceinline__ RotQ<REAL, R> rot_q(const RotDev& g) {
  if constexpr (std::is_same<R, double>::value) {
    if constexpr (REAL)
      return RotShear<double>{g.t, g.b};
    else
      return RotCplx<double>{g.c, g.sr, g.si};
  } else {
    if constexpr (REAL)
      return RotShear<float>{g.ft, g.fb};
    else
      return RotCplx<float>{g.fc, g.fsr, g.fsi};
  }
}

template <int W, int M, bool REAL, class V>
__device__ __forceinline__ void apply_rots(V* v, const RotDev* __restrict__ rots, int nrot) {
  using R = ER<V>;
  if (nrot <= 0) return;
  // the next rotation's parameters are requested before the current one is
  // applied, so the (uniform) load latency overlaps the arithmetic
  RotDev cur = rots[0];
  for (int r = 0; r < nrot; ++r) {
    const RotDev nxt = rots[r + 1 < nrot ? r + 1 : r];
    rot_dispatch<W, M, REAL, V>(cur.p, v, rot_q<REAL, R>(cur));
    cur = nxt;
  }
}

// The rotations of one stage, as the rotation loops see them: the stage's
// rotation list g (a uniform pointer).  The parameters are read straight into
// scalar registers (FP64 values for complex128 elements and row planes, their
// FP32 copies for complex64), one rotation ahead of their use, so no vector
// instruction moves them; the window position selects a scalar branch.
template <class R>
struct RotLane {
  const RotDev* g;
};

template <class T>
__device__ __forceinline__ T uniform_load(const T* p);

// a stage's rotation I, read with scalar loads: the shear parameters (t, b) of
// a real rotation or (c, sr, si) of a complex one, in the element's precision
template <bool REAL, class R>
__device__ __forceinline__ RotQ<REAL, R> rot_params(const RotDev* g, int i) {
  static_assert(offsetof(RotDev, t) == 8 && offsetof(RotDev, b) == 16 && offsetof(RotDev, c) == 24 &&
                    offsetof(RotDev, sr) == 32 && offsetof(RotDev, si) == 40 && offsetof(RotDev, ft) == 48 &&
                    offsetof(RotDev, fb) == 52 && offsetof(RotDev, fc) == 56 && offsetof(RotDev, fsr) == 60 &&
                    offsetof(RotDev, fsi) == 64,
                "scalar parameter loads assume the RotDev layout");
  constexpr bool dbl = std::is_same<R, double>::value;
  constexpr int off = REAL ? (dbl ? 8 : 48) : (dbl ? 24 : 56);
  return uniform_load((const RotQ<REAL, R>*)((const char*)(g + i) + off));
}

// Generic stages: rotation r's position and parameters, loaded one rotation
// ahead; the position selects the code through a scalar branch.
template <int W, int M, bool REAL, class V>
__device__ __forceinline__ void apply_rots_lane(V* v, const RotLane<ER<V>>& rl, int nrot) {
  using R = ER<V>;
  if (nrot <= 0) return;
  RotDev cur = uniform_load(rl.g);
  for (int r = 0; r < nrot; ++r) {
    const RotDev nxt = uniform_load(rl.g + (r + 1 < nrot ? r + 1 : r));
    rot_dispatch<W, M, REAL, V>(cur.p, v, rot_q<REAL, R>(cur));
    cur = nxt;
  }
}

// The rotations of stage shape S, positions fixed at compile time: rotation I
// acts on window position kShapeP[S][I]; its parameters arrive in scalar
// registers, requested while rotation I - 1 is applied.
template <int W, int M, bool REAL, class V, int S, int I>
__device__ __forceinline__ RotQ<REAL, ER<V>> shape_rot(V* v, const RotDev* g, RotQ<REAL, ER<V>> cur) {
  using R = ER<V>;
  constexpr int n = kShapeLen[S];
  const RotQ<REAL, R> nxt = rot_params<REAL, R>(g, I + 1 < n ? I + 1 : I);
  rot_one<W, M, kShapeP[S][I], REAL, V>(v, cur);
  // nothing of a later rotation is scheduled into this one, where it would
  // only hold registers
  __builtin_amdgcn_sched_barrier(0);
  return nxt;
}

template <int W, int M, bool REAL, class V, int S, int... I>
__device__ __forceinline__ void apply_shape(V* v, const RotLane<ER<V>>& rl, std::integer_sequence<int, I...>) {
  using R = ER<V>;
  RotQ<REAL, R> q = rot_params<REAL, R>(rl.g, 0);
  ((q = shape_rot<W, M, REAL, V, S, I>(v, rl.g, q)), ...);
}

// Loads a small struct of uniform, read-only data (descriptor tables written
// before the launch) with scalar memory loads: the address is taken as a
// constant-address-space pointer, so the words arrive in scalar registers
// through the scalar cache, which every block of a launch shares, instead of
// one vector-memory round trip per struct; branches on its fields are scalar
// branches.
template <class T>
__device__ __forceinline__ T uniform_load(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "uniform_load needs whole 32-bit words");
  using cint = const __attribute__((address_space(4))) int;
  T out;
  cint* src = (cint*)p;
  int* dst = (int*)&out;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
  return out;
}

// Block-wide copies between global memory and LDS with U independent loads in
// flight per thread (a plain strided loop waits for every load before the
// next one is issued, which leaves a block with one row in LDS idle for most
// of its staging).
// Marks a loaded value as used here: its load is issued no later than this
// point (and never sunk into a later branch).
__device__ __forceinline__ void keep(const zc64& v) { asm volatile("" ::"v"(v.x), "v"(v.y)); }
__device__ __forceinline__ void keep(const zc128& v) { asm volatile("" ::"v"(v.x), "v"(v.y)); }
__device__ __forceinline__ void keep(const int4& v) { asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w)); }

template <int U, class V>
__device__ __forceinline__ void stage_in(V* __restrict__ dst, const V* __restrict__ src, int len, int tid,
                                         int nthr) {
  for (int e0 = tid; e0 < len; e0 += U * nthr) {
    V t[U];
    // indexes past the end are clamped to the last element: they re-read it
    // and store the same value again, so no load or store is conditional (a
    // conditional store lets the compiler sink its load behind the branch)
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = src[min(e0 + u * nthr, len - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) dst[min(e0 + u * nthr, len - 1)] = t[u];
  }
}

// The same with the destination strided: src[e] goes to dst[e * stride] (a row
// stored as a column of the other layout).
template <int U, class V>
__device__ __forceinline__ void stage_out_strided(V* __restrict__ dst, const V* __restrict__ src, int len,
                                                  int64_t stride, int tid, int nthr) {
  for (int e0 = tid; e0 < len; e0 += U * nthr) {
    V t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = src[min(e0 + u * nthr, len - 1)];
#pragma unroll
    for (int u = 0; u < U; ++u) dst[(int64_t)min(e0 + u * nthr, len - 1) * stride] = t[u];
  }
}

template <class R>
__device__ __forceinline__ typename V2T<R>::type phase_factor(double ang);
template <>
__device__ __forceinline__ zc128 phase_factor<double>(double ang) {
  double s, c;
  sincos(ang, &s, &c);
  return zc128{c, s};
}
template <>
__device__ __forceinline__ zc64 phase_factor<float>(double ang) {
  // the angle stays FP64; reduce to [-pi, pi] before the FP32 sincos
  const double twopi = 6.283185307179586476925286766559;
  double r = ang - twopi * rint(ang / twopi);
  float s, c;
  sincosf((float)r, &s, &c);
  return zc64{c, s};
}

__device__ __forceinline__ double block_sum256(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}


// ---------------------------------------------------------------------------
// a class of an LDS-resident row: load its members into registers, apply the
// stage's rotations, store them back (segment passes and batched tasks)
// ---------------------------------------------------------------------------
// member offsets come four at a time from 16-byte-aligned LDS tables
template <int K>
__device__ __forceinline__ int pick(const int4& q) {
  if constexpr ((K & 3) == 0) return q.x;
  if constexpr ((K & 3) == 1) return q.y;
  if constexpr ((K & 3) == 2) return q.z;
  return q.w;
}

template <int W, int M, bool REAL, class V, int S, int... K>
__device__ __forceinline__ void lds_class(V* __restrict__ row, int cbase, const int* mtl, int moff,
                                          const RotLane<ER<V>>& rl, int nrot, std::integer_sequence<int, K...>) {
  constexpr int C = sizeof...(K);
  constexpr int Q = (C + 3) / 4;
  V v[C];
  {
    int4 q[Q];
    const int4* m4 = (const int4*)(mtl + moff);
#pragma unroll
    for (int i = 0; i < Q; ++i) q[i] = m4[i];
    ((v[K] = row[cbase + pick<K>(q[K >> 2])]), ...);
  }
  if constexpr (S < 0)
    apply_rots_lane<W, M, REAL, V>(v, rl, nrot);
  else
    apply_shape<W, M, REAL, V, S>(v, rl, std::make_integer_sequence<int, kShapeLen[S]>{});
  // nothing of the store-back (the offset reloads in particular) is scheduled
  // into the straight-line rotations, where it would only hold registers
  __builtin_amdgcn_sched_barrier(0);
  // member offsets are re-read from LDS rather than held in registers across
  // the rotations: hiding the table offset from the optimizer forces the reload
  {
    int o = moff;
    asm volatile("" : "+v"(o));
    int4 q[Q];
    const int4* m4 = (const int4*)(mtl + o);
#pragma unroll
    for (int i = 0; i < Q; ++i) q[i] = m4[i];
    ((row[cbase + pick<K>(q[K >> 2])] = v[K]), ...);
  }
}

template <int W, bool REAL, class V, int S = -1, int M = 1>
__device__ __forceinline__ void lds_m(int m, V* row, int cbase, const int* mtl, int moff, const RotLane<ER<V>>& rl,
                                      int nrot) {
  if constexpr (M < W) {
    if (m == M)
      lds_class<W, M, REAL, V, S>(row, cbase, mtl, moff, rl, nrot, std::make_integer_sequence<int, cbinom(W, M)>{});
    else
      lds_m<W, REAL, V, S, M + 1>(m, row, cbase, mtl, moff, rl, nrot);
  }
}

// One Givens stage over the chunks of a window table: wave w takes chunks
// w, w + nwaves, ...; lane l the class code[ch * 64 + l] (negative: none).
// A stage of shape S (uniform; -1 = none) runs that shape's straight-line code.
// A wave's first chunk of a Givens stage (its electron count in the window
// and this lane's class code), requested ahead of the stage.
// (A wave's second chunk, when it has one, is requested with the first: the
// class codes come from global memory, and loading them when the wave reaches
// its second chunk put one memory latency on the stage's critical path.)
struct ChunkAhead {
  int m, m2;
  int code, code2;
};

// TWO = false (row planes, whose register plane leaves no room for the second
// code): only the first chunk is requested ahead.
template <bool TWO = true>
__device__ __forceinline__ ChunkAhead fetch_first_chunk(const SegWinDev& wt, int wave, int lane, int nwaves) {
  ChunkAhead f{1, 1, -1, -1};
  if (wave < wt.n_chunks) {
    f.m = uniform_load(wt.chunk_m + wave);
    f.code = wt.code[wave * 64 + lane];
  }
  if constexpr (TWO) {
    const int w2 = wave + nwaves;
    if (w2 < wt.n_chunks) {
      f.m2 = uniform_load(wt.chunk_m + w2);
      f.code2 = wt.code[w2 * 64 + lane];
    }
  }
  return f;
}

// The rotations of a stage, one per lane (lanes past nrot repeat the last
// one and are never read), loaded without a lane-dependent branch so that the
// load can be issued a stage ahead of its use.
template <class R>
__device__ __forceinline__ RotLane<R> fetch_rot_lane(const RotDev* rots, int nrot, int lane) {
  (void)nrot;
  (void)lane;
  // the same address in every lane; taken through readfirstlane so that the
  // compiler knows it and reads the parameters with scalar loads
  const uint64_t a = (uint64_t)(uintptr_t)rots;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
  return RotLane<R>{(const RotDev*)(uintptr_t)(((uint64_t)hi << 32) | lo)};
}

template <int W, bool REAL, class V, int S>
__device__ __forceinline__ void givens_chunks(V* row, const int* mtl, const SegWinDev& wt, const RotLane<ER<V>>& rl,
                                              int nrot, int wave, int nwaves, int lane, ChunkAhead first) {
  constexpr bool two = !ElemT<V>::plane;  // the second chunk's code was requested ahead
  for (int ch = wave, k = 0; ch < wt.n_chunks; ch += nwaves, ++k) {
    int m = first.m, code = first.code;
    if (two && k == 1) {
      m = first.m2;
      code = first.code2;
    } else if (k > 0) {
      m = uniform_load(wt.chunk_m + ch);
      code = wt.code[ch * 64 + lane];
    }
    // a code holds the class base and the index of its member-offset table
    if (code >= 0) lds_m<W, REAL, V, S>(m, row, code >> kCodeMoffBitsDev, mtl, code & ((1 << kCodeMoffBitsDev) - 1), rl, nrot);
  }
}

template <int W, bool REAL, class V, int S = 0>
__device__ __forceinline__ void givens_stage_v(int shape, V* row, const int* mtl, const SegWinDev& wt,
                                               const RotLane<ER<V>>& rl, int nrot, int wave, int nwaves, int lane,
                                               ChunkAhead first) {
  if constexpr (W == kShapeW && S < kNumShapes) {
    if (shape == S)
      givens_chunks<W, REAL, V, S>(row, mtl, wt, rl, nrot, wave, nwaves, lane, first);
    else
      givens_stage_v<W, REAL, V, S + 1>(shape, row, mtl, wt, rl, nrot, wave, nwaves, lane, first);
  } else {
    givens_chunks<W, REAL, V, -1>(row, mtl, wt, rl, nrot, wave, nwaves, lane, first);
  }
}

// the same on rows of complex amplitudes of scalar type R
template <int W, bool REAL, class R>
__device__ __forceinline__ void givens_stage(int shape, typename V2T<R>::type* row, const int* mtl,
                                             const SegWinDev& wt, const RotLane<R>& rl, int nrot, int wave,
                                             int nwaves, int lane, ChunkAhead first) {
  givens_stage_v<W, REAL, typename V2T<R>::type>(shape, row, mtl, wt, rl, nrot, wave, nwaves, lane, first);
}

__device__ __forceinline__ int parity(uint32_t x) { return __builtin_popcount(x) & 1; }

__device__ __forceinline__ zc128 zmul(zc128 a, zc128 b) {
  return zc128{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

}  // namespace dev
}  // namespace ffx
