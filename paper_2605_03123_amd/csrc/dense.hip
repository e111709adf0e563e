// Dense form of an orbital rotation (Sec. 2.3): Gamma' = C_{n_a}(U_a) Gamma C_{n_b}(U_b)^T with the
// compound matrices C_n(U)[J, I] = det U[J, I] (rows J and columns I the occupied orbitals of two
// configurations, ascending).  It is the plain definition of script-U(U) on the sector, evaluated as
// two complex matrix products on the FP64 matrix cores; the Givens sweeps reach the same result with
// 20 n (N - n) d^2 flops against this form's 16 d^3, so it is built to be measured against them on
// small sectors (d <= a few thousand), not as the default path.
//   * k_compound<n>: one thread per entry, the n x n minor gathered into registers and reduced by
//     Gaussian elimination with partial pivoting in complex FP64.
//   * k_zgemm_mfma: Y = A B (complex128, row-major A and Y, B addressed through two strides so that
//     C^T needs no copy) in 64 x 64 output tiles per block of four waves, 16-deep slices of A and B
//     staged in LDS (real and imaginary parts apart), v_mfma_f64_16x16x4 with the real and imaginary
//     accumulators of each 16 x 16 tile (four products per k step).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dev_common.h"
#include "device.h"

namespace ffx {
namespace dev {

template <int NE>
__global__ __launch_bounds__(256) void k_compound(const uint32_t* __restrict__ masks, int64_t d, int norb,
                                                  const double* __restrict__ U, zc128* __restrict__ C) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int64_t J = idx / d, I = idx - J * d;
  if constexpr (NE == 0) {
    C[idx] = zc128{1.0, 0.0};
  } else {
    int r[NE], c[NE];
    uint32_t mj = masks[J], mi = masks[I];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      r[k] = __builtin_ctz(mj);
      mj &= mj - 1;
      c[k] = __builtin_ctz(mi);
      mi &= mi - 1;
    }
    double ar[NE][NE], ai[NE][NE];
#pragma unroll
    for (int p = 0; p < NE; ++p)
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        ar[p][q] = U[2 * (r[p] * norb + c[q])];
        ai[p][q] = U[2 * (r[p] * norb + c[q]) + 1];
      }
    double dr = 1.0, di = 0.0;
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      // pivot: the largest |a[p][k]| for p >= k; rows swapped by selects (fixed register indices)
      int piv = k;
      double best = ar[k][k] * ar[k][k] + ai[k][k] * ai[k][k];
#pragma unroll
      for (int p = k + 1; p < NE; ++p) {
        const double m = ar[p][k] * ar[p][k] + ai[p][k] * ai[p][k];
        if (m > best) {
          best = m;
          piv = p;
        }
      }
#pragma unroll
      for (int p = k + 1; p < NE; ++p) {
        const bool sw = p == piv;
#pragma unroll
        for (int q = k; q < NE; ++q) {
          const double tr = ar[k][q], ti = ai[k][q];
          ar[k][q] = sw ? ar[p][q] : tr;
          ai[k][q] = sw ? ai[p][q] : ti;
          ar[p][q] = sw ? tr : ar[p][q];
          ai[p][q] = sw ? ti : ai[p][q];
        }
      }
      if (piv != k) {
        dr = -dr;
        di = -di;
      }
      const double pr = ar[k][k], pi = ai[k][k];
      const double nr = dr * pr - di * pi, ni = dr * pi + di * pr;
      dr = nr;
      di = ni;
      if (best == 0.0) break;
      const double inv = 1.0 / best;  // 1 / pivot = conj(pivot) / |pivot|^2
      const double vr = pr * inv, vi = -pi * inv;
#pragma unroll
      for (int p = k + 1; p < NE; ++p) {
        const double fr = ar[p][k] * vr - ai[p][k] * vi, fi = ar[p][k] * vi + ai[p][k] * vr;
#pragma unroll
        for (int q = k + 1; q < NE; ++q) {
          ar[p][q] -= fr * ar[k][q] - fi * ai[k][q];
          ai[p][q] -= fr * ai[k][q] + fi * ar[k][q];
        }
      }
    }
    C[idx] = zc128{dr, di};
  }
}

void compound_matrix(const uint32_t* masks, int64_t d, int n, int norb, const double* U, void* C, hipStream_t s) {
  const dim3 g((unsigned)((d * d + 255) / 256)), b(256);
  zc128* out = (zc128*)C;
  switch (n) {
    case 0: hipLaunchKernelGGL(k_compound<0>, g, b, 0, s, masks, d, norb, U, out); break;
    case 1: hipLaunchKernelGGL(k_compound<1>, g, b, 0, s, masks, d, norb, U, out); break;
    case 2: hipLaunchKernelGGL(k_compound<2>, g, b, 0, s, masks, d, norb, U, out); break;
    case 3: hipLaunchKernelGGL(k_compound<3>, g, b, 0, s, masks, d, norb, U, out); break;
    case 4: hipLaunchKernelGGL(k_compound<4>, g, b, 0, s, masks, d, norb, U, out); break;
    case 5: hipLaunchKernelGGL(k_compound<5>, g, b, 0, s, masks, d, norb, U, out); break;
    case 6: hipLaunchKernelGGL(k_compound<6>, g, b, 0, s, masks, d, norb, U, out); break;
    case 7: hipLaunchKernelGGL(k_compound<7>, g, b, 0, s, masks, d, norb, U, out); break;
    case 8: hipLaunchKernelGGL(k_compound<8>, g, b, 0, s, masks, d, norb, U, out); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// complex128 GEMM on the FP64 matrix cores.  v_mfma_f64_16x16x4: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[l / 16 + 4 t][l % 16],
// t = 0..3.  Re Y += Ar Br - Ai Bi and Im Y += Ar Bi + Ai Br: four products
// into two accumulators per 16 x 16 tile.
// ---------------------------------------------------------------------------
typedef double zg_d4 __attribute__((ext_vector_type(4)));
constexpr int kGT = 64;  // output tile edge
constexpr int kGK = 16;  // k slice

__global__ __launch_bounds__(256) void k_zgemm_mfma(const zc128* __restrict__ A, int64_t lda,
                                                    const zc128* __restrict__ B, int64_t sbk, int64_t sbn,
                                                    zc128* __restrict__ Y, int64_t ldy, int M, int N, int K) {
  __shared__ double sar[kGK][kGT + 1], sai[kGK][kGT + 1];  // A slice, [k][m]
  __shared__ double sbr[kGK][kGT + 1], sbi[kGK][kGT + 1];  // B slice, [k][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const bool bk_fast = sbk == 1;
  zg_d4 re[2][2], im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      re[i][j] = zg_d4{0.0, 0.0, 0.0, 0.0};
      im[i][j] = re[i][j];
    }
  for (int k0 = 0; k0 < K; k0 += kGK) {
    zc128 av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      const int am = e >> 4, ak = e & 15;  // k fastest: 16 consecutive elements of a row of A
      const int gm = m0 + am, gk = k0 + ak;
      av[u] = (gm < M && gk < K) ? A[(int64_t)gm * lda + gk] : zc128{0.0, 0.0};
      const int bk = bk_fast ? (e & 15) : (e >> 6), bn = bk_fast ? (e >> 4) : (e & 63);
      const int hk = k0 + bk, hn = n0 + bn;
      bv[u] = (hk < K && hn < N) ? B[(int64_t)hk * sbk + (int64_t)hn * sbn] : zc128{0.0, 0.0};
    }
    __syncthreads();  // the previous slice's readers are done
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      sar[e & 15][e >> 4] = av[u].x;
      sai[e & 15][e >> 4] = av[u].y;
      const int bk = bk_fast ? (e & 15) : (e >> 6), bn = bk_fast ? (e >> 4) : (e & 63);
      sbr[bk][bn] = bv[u].x;
      sbi[bk][bn] = bv[u].y;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      const int k = kk + (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const double ar = sar[k][wm + 16 * i + (lane & 15)], ai = sai[k][wm + 16 * i + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double br = sbr[k][wn + 16 * j + (lane & 15)], bi = sbi[k][wn + 16 * j + (lane & 15)];
          re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, re[i][j], 0, 0, 0);
          re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, re[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, im[i][j], 0, 0, 0);
          im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, im[i][j], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int gm = m0 + wm + 16 * i + (lane >> 4) + 4 * t, gn = n0 + wn + 16 * j + (lane & 15);
        if (gm < M && gn < N) Y[(int64_t)gm * ldy + gn] = zc128{re[i][j][t], im[i][j][t]};
      }
}

void zgemm_mfma(const void* A, int64_t lda, const void* B, int64_t sbk, int64_t sbn, void* Y, int64_t ldy, int M,
                int N, int K, hipStream_t s) {
  const dim3 g((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT)), b(256);
  hipLaunchKernelGGL(k_zgemm_mfma, g, b, 0, s, (const zc128*)A, lda, (const zc128*)B, sbk, sbn, (zc128*)Y, ldy, M, N,
                     K);
}

}  // namespace dev
}  // namespace ffx
