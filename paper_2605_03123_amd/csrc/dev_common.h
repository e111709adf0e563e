// Device-side helpers shared by the HIP translation units of libffx:
// complex amplitude types, compile-time pattern / pair tables of a window, the
// register-resident Givens application, phase factors and block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
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

// x' = c x + s y, y' = -conj(s) x + c y on one member pair (A, B)
template <int A, int B, bool REAL, class R>
__device__ __forceinline__ void rot_pair(typename V2T<R>::type* v, R c, R sr, R si) {
  using V = typename V2T<R>::type;
  V x = v[A], y = v[B];
  V nx, ny;
  if constexpr (REAL) {
    nx.x = c * x.x + sr * y.x;
    nx.y = c * x.y + sr * y.y;
    ny.x = c * y.x - sr * x.x;
    ny.y = c * y.y - sr * x.y;
  } else {
    nx.x = c * x.x + sr * y.x - si * y.y;
    nx.y = c * x.y + sr * y.y + si * y.x;
    ny.x = c * y.x - sr * x.x - si * x.y;
    ny.y = c * y.y - sr * x.y + si * x.x;
  }
  v[A] = nx;
  v[B] = ny;
}

// every member pair of rotation P, expanded at compile time so that the
// register array is only ever indexed by constants
template <int W, int M, int P, bool REAL, class R, int... I>
__device__ __forceinline__ void rot_pairs(typename V2T<R>::type* v, R c, R sr, R si,
                                          std::integer_sequence<int, I...>) {
  constexpr Pairs<W, M, P> pr{};
  (rot_pair<pr.a[I], pr.b[I], REAL, R>(v, c, sr, si), ...);
}

template <int W, int M, int P, bool REAL, class R>
__device__ __forceinline__ void rot_one(typename V2T<R>::type* v, R c, R sr, R si) {
  rot_pairs<W, M, P, REAL, R>(v, c, sr, si, std::make_integer_sequence<int, Pairs<W, M, P>::NP>{});
}

template <int W, int M, int P, bool REAL, class R>
__device__ __forceinline__ void rot_case(typename V2T<R>::type* v, R c, R sr, R si) {
  if constexpr (P < W - 1) rot_one<W, M, P, REAL, R>(v, c, sr, si);
}

// one uniform jump per rotation (a dense switch lowers to a jump table)
template <int W, int M, bool REAL, class R>
__device__ __forceinline__ void rot_dispatch(int p, typename V2T<R>::type* v, R c, R sr, R si) {
  static_assert(W <= 8, "window wider than the dispatch table");
  switch (p) {
    case 0: rot_case<W, M, 0, REAL, R>(v, c, sr, si); break;
    case 1: rot_case<W, M, 1, REAL, R>(v, c, sr, si); break;
    case 2: rot_case<W, M, 2, REAL, R>(v, c, sr, si); break;
    case 3: rot_case<W, M, 3, REAL, R>(v, c, sr, si); break;
    case 4: rot_case<W, M, 4, REAL, R>(v, c, sr, si); break;
    case 5: rot_case<W, M, 5, REAL, R>(v, c, sr, si); break;
    case 6: rot_case<W, M, 6, REAL, R>(v, c, sr, si); break;
    default: break;
  }
}

template <int W, int M, bool REAL, class R>
__device__ __forceinline__ void apply_rots(typename V2T<R>::type* v, const RotDev* __restrict__ rots,
                                           int nrot) {
  if (nrot <= 0) return;
  // the next rotation's parameters are requested before the current one is
  // applied, so the (uniform) load latency overlaps the arithmetic
  RotDev cur = rots[0];
  for (int r = 0; r < nrot; ++r) {
    const RotDev nxt = rots[r + 1 < nrot ? r + 1 : r];
    rot_dispatch<W, M, REAL, R>(cur.p, v, (R)cur.c, (R)cur.sr, (R)cur.si);
    cur = nxt;
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


}  // namespace dev
}  // namespace ffx
