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

#include <algorithm>
#include <utility>

#include "dev_common.h"
#include "device.h"

namespace ffx {
namespace dev {

// 12 waves per block (3 per SIMD): the widest register windows (W = 7 at
// complex64, W = 6 at complex128) fit in the 168 registers this leaves a lane;
// narrower windows fit in 128 registers and run 16 waves
template <int W, class R>
constexpr int seg_threads() {
  return (sizeof(R) == 4 ? W <= 6 : W <= 5) ? 1024 : 768;
}

// The rotation on the orbital pair that straddles the segment window, for
// the cnt strings own[0 .. cnt) of this segment and their partners peer[0 ..
// cnt) in another segment of the same row (read from the pass's source, which
// the pass does not write): role 0: own = x, x' = c x + s y; role 1: own = y,
// y' = c y - conj(s) x.  The first kCrossU partners of each thread are loaded
// together with the segment itself (cross_fetch, before the barrier that
// completes the segment); cross_apply then rotates, loading any further
// partners directly.
constexpr int kCrossU = 8;

__device__ const int4 kZeroWords = {0, 0, 0, 0};

// The block's row segment, the member-offset tables (int4 words) and the
// first kCrossU crossing partners per thread, requested in one straight-line
// batch before any is used: every thread issues all its loads (clamped to the
// last valid element, pointers chosen without branches), then stores the
// segment and the tables to LDS; the partners stay in registers (xt).  Further
// batches run only for segments longer than UR * nthr or tables longer than
// UM * nthr words.
// stride: distance between consecutive elements of the row in src and peer
// (1, or the row count of a gathering pass, whose src is the other layout).
template <int UR, int UM, class V>
__device__ __forceinline__ void stage_segment(V* __restrict__ row, const V* __restrict__ src, int len,
                                              int4* __restrict__ mt, const int4* mtg, int n4, const V* peer,
                                              int pcnt, V* xt, int tid, int nthr, int64_t stride) {
  const int4* pm = n4 > 0 ? mtg : &kZeroWords;
  const int pn4 = max(n4, 1);
  const V* pp = pcnt > 0 ? peer : src;
  const int pc = max(pcnt, 1);
  V t[UR];
  int4 q[UM];
#pragma unroll
  for (int u = 0; u < UR; ++u) t[u] = src[(int64_t)min(tid + u * nthr, len - 1) * stride];
#pragma unroll
  for (int u = 0; u < UM; ++u) q[u] = pm[min(tid + u * nthr, pn4 - 1)];
#pragma unroll
  for (int u = 0; u < kCrossU; ++u) xt[u] = pp[(int64_t)min(tid + u * nthr, pc - 1) * stride];
#pragma unroll
  for (int u = 0; u < UR; ++u) keep(t[u]);
#pragma unroll
  for (int u = 0; u < UM; ++u) keep(q[u]);
#pragma unroll
  for (int u = 0; u < UR; ++u)
    if (tid + u * nthr < len) row[tid + u * nthr] = t[u];
#pragma unroll
  for (int u = 0; u < UM; ++u)
    if (tid + u * nthr < n4) mt[tid + u * nthr] = q[u];
  for (int e = tid + UR * nthr; e < len; e += nthr) row[e] = src[(int64_t)e * stride];
  for (int e = tid + UM * nthr; e < n4; e += nthr) mt[e] = mtg[e];
}

template <class R>
__device__ __forceinline__ typename V2T<R>::type cross_rot(typename V2T<R>::type a, typename V2T<R>::type b, R c,
                                                           R sgn, R sr, R si) {
  // own' = c own + sgn * s' peer, s' = s (role 0) or conj(s) (role 1)
  typename V2T<R>::type o;
  o.x = c * a.x + sgn * (sr * b.x - si * b.y);
  o.y = c * a.y + sgn * (sr * b.y + si * b.x);
  return o;
}

template <class R>
__device__ __forceinline__ void cross_apply(typename V2T<R>::type* own, const typename V2T<R>::type* t,
                                            const typename V2T<R>::type* peer, int cnt, int role, double cd,
                                            double srd, double sid, int tid, int nthr, int64_t stride) {
  const R c = (R)cd, sr = (R)srd, si = role == 0 ? (R)sid : -(R)sid;
  const R sgn = role == 0 ? R(1) : R(-1);
#pragma unroll
  for (int u = 0; u < kCrossU; ++u) {
    const int e = tid + u * nthr;
    if (e < cnt) own[e] = cross_rot<R>(own[e], t[u], c, sgn, sr, si);
  }
  for (int e = tid + kCrossU * nthr; e < cnt; e += nthr)
    own[e] = cross_rot<R>(own[e], peer[(int64_t)e * stride], c, sgn, sr, si);
}

// Row-dependent part of a diagonal stage, computed by the whole block before
// the stage touches any element: the cross weights w[q] = sum_{p in row} C[p][q]
// (the row's masked C is staged in the table area, one load per thread, all in
// flight at once, then summed over p in a fixed order), the row value A[r], the
// row's phase factor (phase stages; with a cross term it is folded into the
// first byte table), and the byte tables of the cross term: complex factors for
// phase stages, real sums otherwise.  Ends with a block barrier.
struct DiagRow {
  double arow;
  zc128 rowf;
  bool cross;
};

__device__ __forceinline__ DiagRow diag_stage_tables(const StageDev& st, const SegPassDev& P, int64_t r,
                                                     uint32_t rmask, zc128* ez, double* wq, int tid, int nthr,
                                                     int nbytes) {
  double* tab = (double*)ez;
  DiagRow dr;
  dr.cross = st.C != nullptr;
  const int nn = P.norb * P.norb;
  if (dr.cross) {
    for (int i = tid; i < nn; i += nthr) tab[i] = ((rmask >> (i / P.norb)) & 1) ? st.C[i] : 0.0;
    __syncthreads();
  }
  if (tid < P.norb) {
    double w = 0.0;
    if (dr.cross)
      for (int p = 0; p < P.norb; ++p) w += tab[p * P.norb + tid];
    wq[tid] = w;
  }
  __syncthreads();
  dr.arow = st.A ? st.A[r] : 0.0;
  dr.rowf = zc128{1.0, 0.0};
  if (st.type == ST_PHASE) {
    double grow = 0.0;
    if (st.drow)
      for (int p = 0; p < P.norb; ++p)
        if ((rmask >> p) & 1) grow += st.drow[p];
    dr.rowf = phase_factor<double>(st.scale * dr.arow + grow);
    if (parity(rmask & st.sign_row)) {
      dr.rowf.x = -dr.rowf.x;
      dr.rowf.y = -dr.rowf.y;
    }
  }
  if (dr.cross) {
    for (int i = tid; i < nbytes * 256; i += nthr) {
      const int k = i >> 8, b = i & 255;
      double v = 0.0;
      for (int q = 0; q < 8; ++q)
        if (((b >> q) & 1) && 8 * k + q < P.norb) v += wq[8 * k + q];
      if (st.type == ST_PHASE) {
        const zc128 e = phase_factor<double>(st.scale * v);
        ez[i] = k == 0 ? zmul(dr.rowf, e) : e;
      } else {
        tab[i] = v;
      }
    }
  }
  __syncthreads();
  return dr;
}

template <int W, bool REAL, class R>
__global__ __launch_bounds__((seg_threads<W, R>())) void k_seg_pass(SegPassDev P) {
  using V = typename V2T<R>::type;
  extern __shared__ __align__(16) char smem[];
  V* row = (V*)smem;
  zc128* ez = (zc128*)(smem + P.lds_row_bytes);      // 4 x 256 complex byte factors
  double* tab = (double*)ez;                          // (or 4 x 256 real byte sums)
  int* mtl = (int*)(ez + 4 * 256);                    // member offsets of one window
  double* wq = (double*)(mtl + ((P.max_mt + 3) & ~3)); // 32 cross weights
  double* red = wq + 32;                               // block reduction scratch

  int si;
  int64_t r;
  if (P.xcd_rows > 0) {
    const int64_t k = blockIdx.x >> 3;
    r = (int64_t)(blockIdx.x & 7) * P.xcd_rows + k / P.n_seg;
    si = (int)(k % P.n_seg);
    if (r >= P.n_rows) return;  // the whole block: the grid rounds rows up to 8 XCDs
  } else {
    si = (int)(blockIdx.x % P.n_seg);
    r = blockIdx.x / P.n_seg;
  }
  const int64_t blk = r * P.n_seg + si;
  const SegDev sg = uniform_load(P.segs + si);
  const int nthr = blockDim.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave: loops over chunks stay scalar
  const int nwaves = nthr >> 6;

  // row r of this layout: contiguous, or column r of the other layout
  const int64_t stride = P.gather ? P.n_rows : 1;
  const V* src = P.gather ? (const V*)P.src + r + (int64_t)sg.off * P.n_rows
                          : (const V*)P.src + r * P.row_len + sg.off;
  const bool xrot = P.cross && sg.cross_cnt > 0;
  const V* peer = P.gather ? (const V*)P.src + r + (int64_t)sg.cross_peer * P.n_rows
                           : (const V*)P.src + r * P.row_len + sg.cross_peer;
  V xt[kCrossU];
  // (the member-offset table of every window is a whole number of int4 words)
  stage_segment<sizeof(V) == 8 ? 13 : 9, 2>(row, src, sg.len, (int4*)mtl, (const int4*)sg.mt_all,
                                            sg.n_mt_all >> 2, peer, xrot ? sg.cross_cnt : 0, xt, tid, nthr, stride);
  __syncthreads();
  if (xrot) {
    cross_apply<R>(row + sg.cross_lo, xt, peer, sg.cross_cnt, sg.cross_role, P.cross_c, P.cross_sr, P.cross_si,
                   tid, nthr, stride);
    __syncthreads();
  }

  const uint32_t rmask = P.row_masks[r];
  const uint32_t* cmask = P.col_masks + sg.off;
  const int nbytes = (P.norb + 7) >> 3;
  double acc = 0.0;

  // the vector-memory data of a Givens stage (its rotations, the wave's first
  // class codes) is requested one stage ahead, so that its latency overlaps the
  // stage before; descriptors come through the scalar cache
  RotLane<R> rl_next{nullptr};
  ChunkAhead fc_next{1, 1, -1, -1};
  auto fetch = [&](int s) {
    const StageDev st = uniform_load(P.stages + s);
    if (st.type == ST_GIVENS) {
      rl_next = fetch_rot_lane<R>(st.rots, st.nrot, lane);
      fc_next = fetch_first_chunk(uniform_load(sg.win + st.a), wave, lane, nwaves);
    }
  };
  if (P.n_stages > 0) fetch(0);
  for (int s = 0; s < P.n_stages; ++s) {
    const StageDev st = uniform_load(P.stages + s);
    const RotLane<R> rl = rl_next;
    const ChunkAhead fc = fc_next;
    if (s + 1 < P.n_stages) fetch(s + 1);
    if (st.type == ST_GIVENS) {
      const SegWinDev wt = uniform_load(sg.win + st.a);
      givens_stage<W, REAL, R>(st.shape, row, mtl, wt, rl, st.nrot, wave, nwaves, lane, fc);
    } else {
      const DiagRow dr = diag_stage_tables(st, P, r, rmask, ez, wq, tid, nthr, nbytes);
      const bool cross = dr.cross;
      const double arow = dr.arow;
      zc128 rowf = dr.rowf;
      // U elements per thread at a time (a whole segment per batch for the
      // usual block sizes): their column masks and tables are all requested
      // before the first is used
      constexpr int U = sizeof(V) == 8 ? 10 : 9;
      if (st.type == ST_PHASE) {
        if (cross) rowf = zc128{1.0, 0.0};
        const zc128* colf = st.colf ? (const zc128*)st.colf + sg.off : nullptr;
        const uint32_t sgn = st.sign_col;
        const bool use_cm = cross || sgn != 0;
        // signs only: negate where the row and column parities differ
        const bool signs_only = !cross && !colf && !st.A && !st.drow;
        const int rneg = rowf.x < 0.0;
        const zc128 one{1.0, 0.0};
        for (int e0 = tid; e0 < sg.len; e0 += U * nthr) {
          uint32_t cm[U];
          zc128 cf[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = min(e0 + u * nthr, sg.len - 1);
            cm[u] = use_cm ? cmask[e] : 0u;
            cf[u] = colf ? colf[e] : one;
          }
#pragma unroll
          for (int u = 0; u < U; ++u) asm volatile("" ::"v"(cm[u]), "v"(cf[u].x), "v"(cf[u].y));
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = e0 + u * nthr;
            if (e >= sg.len) continue;
            if (signs_only) {
              if (parity(cm[u] & sgn) != rneg) {
                V y = row[e];
                y.x = -y.x;
                y.y = -y.y;
                row[e] = y;
              }
              continue;
            }
            zc128 f = colf ? zmul(rowf, cf[u]) : rowf;
            if (cross)
              for (int k = 0; k < nbytes; ++k) f = zmul(f, ez[(k << 8) | ((cm[u] >> (8 * k)) & 255)]);
            if (parity(cm[u] & sgn)) {
              f.x = -f.x;
              f.y = -f.y;
            }
            V y = row[e];
            V o;
            o.x = (R)((double)y.x * f.x - (double)y.y * f.y);
            o.y = (R)((double)y.x * f.y + (double)y.y * f.x);
            row[e] = o;
          }
        }
      } else {
        const double* Bs = st.B ? st.B + sg.off : nullptr;
        for (int e0 = tid; e0 < sg.len; e0 += U * nthr) {
          uint32_t cm[U];
          double fb[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = min(e0 + u * nthr, sg.len - 1);
            cm[u] = cross ? cmask[e] : 0u;
            fb[u] = Bs ? Bs[e] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < U; ++u) asm volatile("" ::"v"(cm[u]), "v"(fb[u]));
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = e0 + u * nthr;
            if (e < sg.len) {
              double f = arow + fb[u];
              if (cross)
                for (int k = 0; k < nbytes; ++k) f += tab[(k << 8) | ((cm[u] >> (8 * k)) & 255)];
              V y = row[e];
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
      }
    }
    __syncthreads();
  }

  if (P.mode != SEG_NONE) {
    // row r of this layout, or (scatter) column r of the other one
    const int64_t ostride = P.scatter ? P.n_rows : 1;
    V* dst = P.scatter ? (V*)P.dst + r + (int64_t)sg.off * P.n_rows : (V*)P.dst + r * P.row_len + sg.off;
    if (P.mode == SEG_STORE) {
      if (P.scatter)
        stage_out_strided<128 / sizeof(V)>(dst, row, sg.len, ostride, tid, nthr);
      else
        stage_in<128 / sizeof(V)>(dst, row, sg.len, tid, nthr);
    } else {
      for (int e = tid; e < sg.len; e += nthr) {
        V a = dst[e * ostride], b = row[e];
        a.x += b.x;
        a.y += b.y;
        dst[e * ostride] = a;
      }
    }
  }
  if (P.partials) {
    // fixed-order block reduction: wave sums, then thread 0 adds them in order
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

// ---------------------------------------------------------------------------
// Row planes.  A complex128 row that exceeds LDS, but whose real parts fit,
// is held as two planes when every Givens rotation of the pass is real: a real
// rotation matrix acts on the real and imaginary parts of the amplitudes alike
// and independently, so each run of consecutive Givens stages is applied to
// the plane in LDS, the planes are swapped, and the run is applied to the
// other.  The other plane stays in registers: thread t holds the parts of
// elements t, t + nthr, t + 2 nthr, ...  Diagonal stages combine the two parts
// of each element in the thread that holds its register part.  Where the real
// parts of a whole row fit, the row is one segment and no rotation crosses a
// segment: one pass per visit.  Longer rows are split, as in the segment pass,
// into segments of the strings that share their highest orbitals (the
// rotations on those orbitals run as whole-spin window passes between plane
// passes); each block holds one segment of one row.
// ---------------------------------------------------------------------------
// Block sizes: 768 threads hold 17 register parts each (rows of up to 13 056
// amplitudes, 168 registers a lane, 3 waves per SIMD; the default, 5 % faster
// on the DF step at 16 orbitals) or 512 threads 26 parts (13 312 amplitudes,
// 200 registers, 2 waves per SIMD).
template <int NT>
constexpr int plane_regs() {
  return NT == 512 ? 26 : 17;
}

int seg_pass_plane_max_len(int threads) { return threads * (threads == 512 ? plane_regs<512>() : plane_regs<768>()); }

// Givens stages [s0, s1) of a plane pass on the LDS plane; each stage's
// rotations and the wave's first class codes are requested one stage ahead.
template <int W>
__device__ __forceinline__ void plane_givens_run(const SegPassDev& P, const SegDev& sg, re128* pl, const int* mtl,
                                                 int s0, int s1, int wave, int nwaves, int lane) {
  StageDev st = uniform_load(P.stages + s0);
  RotLane<double> rl_next = fetch_rot_lane<double>(st.rots, st.nrot, lane);
  ChunkAhead fc_next = fetch_first_chunk<false>(uniform_load(sg.win + st.a), wave, lane, nwaves);
  for (int s = s0; s < s1; ++s) {
    st = uniform_load(P.stages + s);
    const RotLane<double> rl = rl_next;
    const ChunkAhead fc = fc_next;
    if (s + 1 < s1) {
      const StageDev nx = uniform_load(P.stages + s + 1);
      rl_next = fetch_rot_lane<double>(nx.rots, nx.nrot, lane);
      fc_next = fetch_first_chunk<false>(uniform_load(sg.win + nx.a), wave, lane, nwaves);
    }
    const SegWinDev wt = uniform_load(sg.win + st.a);
    givens_stage_v<W, true, re128>(st.shape, pl, mtl, wt, rl, st.nrot, wave, nwaves, lane, fc);
    __syncthreads();
  }
}

// SEGS: rows split into segments (else one segment, the whole row, at offset 0)
template <int W, int NT, bool SEGS>
__global__ __launch_bounds__(NT) void k_seg_pass_planes(SegPassDev P) {
  constexpr int kPlaneRegs = plane_regs<NT>();
  extern __shared__ __align__(16) char smem[];
  re128* pl = (re128*)smem;                            // the LDS plane
  zc128* ez = (zc128*)(smem + P.lds_row_bytes);        // 4 x 256 complex byte factors
  double* tab = (double*)ez;                           // (or 4 x 256 real byte sums)
  int* mtl = (int*)(ez + 4 * 256);                     // member offsets of every window
  double* wq = (double*)(mtl + ((P.max_mt + 3) & ~3)); // 32 cross weights
  double* red = wq + 32;                               // block reduction scratch

  // block -> (row, segment) as in the segment pass
  int si = 0;
  int64_t r;
  if constexpr (SEGS) {
    if (P.xcd_rows > 0) {
      const int64_t k = blockIdx.x >> 3;
      r = (int64_t)(blockIdx.x & 7) * P.xcd_rows + k / P.n_seg;
      si = (int)(k % P.n_seg);
      if (r >= P.n_rows) return;  // the whole block: the grid rounds rows up to 8 XCDs
    } else {
      si = (int)(blockIdx.x % P.n_seg);
      r = blockIdx.x / P.n_seg;
    }
  } else {
    if (P.xcd_rows > 0) {
      r = (int64_t)(blockIdx.x & 7) * P.xcd_rows + (blockIdx.x >> 3);
      if (r >= P.n_rows) return;
    } else {
      r = blockIdx.x;
    }
  }
  const int64_t blk = SEGS ? r * P.n_seg + si : r;
  const SegDev sg = uniform_load(P.segs + si);
  const int off = SEGS ? sg.off : 0;  // the segment's first column
  const int len = sg.len;
  const int nthr = blockDim.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wave: loops over chunks stay scalar
  const int nwaves = nthr >> 6;
  const int64_t stride = P.gather ? P.n_rows : 1;
  const zc128* src = P.gather ? (const zc128*)P.src + r + (int64_t)off * P.n_rows
                              : (const zc128*)P.src + r * P.row_len + off;

  // the row: every load in flight before the first is used; real parts to the
  // LDS plane, imaginary parts to registers; then the member-offset tables
  double rp[kPlaneRegs];
  {
    zc128 t[kPlaneRegs];
#pragma unroll
    for (int k = 0; k < kPlaneRegs; ++k) t[k] = src[(int64_t)min(tid + k * nthr, len - 1) * stride];
#pragma unroll
    for (int k = 0; k < kPlaneRegs; ++k) keep(t[k]);
#pragma unroll
    for (int k = 0; k < kPlaneRegs; ++k) {
      const int e = tid + k * nthr;
      if (e < len) pl[e].x = t[k].x;
      rp[k] = t[k].y;
    }
  }
  for (int e = tid; e < (sg.n_mt_all >> 2); e += nthr) ((int4*)mtl)[e] = ((const int4*)sg.mt_all)[e];
  __syncthreads();
  bool lds_re = true;  // the LDS plane holds the real parts (the same in every thread)

  const uint32_t rmask = P.row_masks[r];
  const uint32_t* cmask = P.col_masks + off;
  const int nbytes = (P.norb + 7) >> 3;
  double acc = 0.0;
  int s = 0;
  while (s < P.n_stages) {
    const StageDev st = uniform_load(P.stages + s);
    if (st.type == ST_GIVENS) {
      int s1 = s + 1;
      while (s1 < P.n_stages && uniform_load(P.stages + s1).type == ST_GIVENS) ++s1;
      plane_givens_run<W>(P, sg, pl, mtl, s, s1, wave, nwaves, lane);
      // swap the planes: the register plane into LDS and back
#pragma unroll
      for (int k = 0; k < kPlaneRegs; ++k) {
        int e = tid + k * nthr;
        asm volatile("" : "+v"(e));  // recomputed here: hoisted, 26 such offsets would stay live across stages
        if (e < len) {
          const double x = pl[e].x;
          pl[e].x = rp[k];
          rp[k] = x;
        }
      }
      __syncthreads();
      lds_re = !lds_re;
      plane_givens_run<W>(P, sg, pl, mtl, s, s1, wave, nwaves, lane);
      s = s1;
      continue;
    }
    const DiagRow dr = diag_stage_tables(st, P, r, rmask, ez, wq, tid, nthr, nbytes);
    const bool cross = dr.cross;
    if (st.type == ST_PHASE) {
      const zc128 rowf = cross ? zc128{1.0, 0.0} : dr.rowf;
      const zc128* colf = st.colf ? (const zc128*)st.colf + off : nullptr;
      const uint32_t sgn = st.sign_col;
      const bool use_cm = cross || sgn != 0;
#pragma unroll
      for (int k = 0; k < kPlaneRegs; ++k) {
        int e = tid + k * nthr;
        asm volatile("" : "+v"(e));  // recomputed per element (see the swap)
        if (e >= len) continue;
        const uint32_t cm = use_cm ? cmask[e] : 0u;
        zc128 f = colf ? zmul(rowf, colf[e]) : rowf;
        if (cross)
          for (int b = 0; b < nbytes; ++b) f = zmul(f, ez[(b << 8) | ((cm >> (8 * b)) & 255)]);
        if (parity(cm & sgn)) {
          f.x = -f.x;
          f.y = -f.y;
        }
        const double a = pl[e].x, q = rp[k];
        const double re = lds_re ? a : q, im = lds_re ? q : a;
        const double nre = re * f.x - im * f.y, nim = re * f.y + im * f.x;
        pl[e].x = lds_re ? nre : nim;
        rp[k] = lds_re ? nim : nre;
      }
    } else {
      const double* Bs = st.B ? st.B + off : nullptr;
#pragma unroll
      for (int k = 0; k < kPlaneRegs; ++k) {
        int e = tid + k * nthr;
        asm volatile("" : "+v"(e));  // recomputed per element (see the swap)
        if (e >= len) continue;
        double f = dr.arow + (Bs ? Bs[e] : 0.0);
        if (cross) {
          const uint32_t cm = cmask[e];
          for (int b = 0; b < nbytes; ++b) f += tab[(b << 8) | ((cm >> (8 * b)) & 255)];
        }
        if (st.type == ST_SCALE) {
          pl[e].x *= f;
          rp[k] *= f;
        } else {
          const double a = pl[e].x, q = rp[k];
          acc += f * (a * a + q * q);
        }
      }
    }
    __syncthreads();
    ++s;
  }

  if (P.mode != SEG_NONE) {
    // row r of this layout, or (scatter) column r of the other one
    const int64_t ostride = P.scatter ? P.n_rows : 1;
    zc128* dst = P.scatter ? (zc128*)P.dst + r + (int64_t)off * P.n_rows : (zc128*)P.dst + r * P.row_len + off;
#pragma unroll
    for (int k = 0; k < kPlaneRegs; ++k) {
      const int e = tid + k * nthr;
      if (e < len) {
        const double a = pl[e].x, q = rp[k];
        zc128 v = lds_re ? zc128{a, q} : zc128{q, a};
        if (P.mode == SEG_ACCUM) {
          const zc128 o = dst[e * ostride];
          v.x += o.x;
          v.y += o.y;
        }
        dst[e * ostride] = v;
      }
    }
  }
  if (P.partials) {
    // fixed-order block reduction: wave sums, then thread 0 adds them in order
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

template <int W, int NT, bool SEGS>
static void launch_planes(const SegPassDev& p, size_t lds, hipStream_t s) {
  auto k = k_seg_pass_planes<W, NT, SEGS>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  const int64_t blocks = p.xcd_rows > 0 ? 8 * p.xcd_rows * p.n_seg : p.n_rows * p.n_seg;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(NT), lds, s, p);
}

// rows split into segments only at window width 6 (the plan builds no
// narrower segmented plane set)
template <int NT>
static void planes_w(int W, const SegPassDev& p, size_t lds, hipStream_t s) {
  if (p.n_seg > 1) {
    if (W == 6) launch_planes<6, NT, true>(p, lds, s);
    return;
  }
  switch (W) {
    case 4: launch_planes<4, NT, false>(p, lds, s); break;
    case 5: launch_planes<5, NT, false>(p, lds, s); break;
    case 6: launch_planes<6, NT, false>(p, lds, s); break;
    default: break;
  }
}

void seg_pass_planes(int W, int threads, const SegPassDev& p, size_t lds, hipStream_t s) {
  if (threads == 768)
    planes_w<768>(W, p, lds, s);
  else
    planes_w<512>(W, p, lds, s);
}

__global__ void k_column_factors(const uint32_t* __restrict__ masks, int64_t n, const double* __restrict__ B,
                                 double scale, const double* __restrict__ delta, uint32_t sign,
                                 zc128* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t m = masks[i];
  double ang = B ? scale * B[i] : 0.0;
  if (delta) {
    uint32_t x = m;
    while (x) {
      ang += delta[__builtin_ctz(x)];
      x &= x - 1;
    }
  }
  zc128 f = phase_factor<double>(ang);
  if (parity(m & sign)) {
    f.x = -f.x;
    f.y = -f.y;
  }
  out[i] = f;
}

void column_factors(const uint32_t* masks, int64_t n, const double* B, double scale, const double* delta,
                    uint32_t sign, double* colf, hipStream_t s) {
  hipLaunchKernelGGL(k_column_factors, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, masks, n, B, scale,
                     delta, sign, (zc128*)colf);
}

size_t seg_pass_lds(bool c64, int max_len, int max_mt) {
  size_t row = (size_t)max_len * (c64 ? 8 : 16);
  row = (row + 15) & ~(size_t)15;
  return row + 4 * 256 * sizeof(zc128) + (size_t)((max_mt + 3) & ~3) * sizeof(int) + (32 + 16) * sizeof(double);
}

int seg_pass_threads(bool c64, int W, int requested) {
  const int cap = c64 ? (W <= 6 ? seg_threads<6, float>() : seg_threads<7, float>())
                      : (W <= 5 ? seg_threads<5, double>() : seg_threads<6, double>());
  return std::min(requested, cap);
}

template <int W, bool REAL, class R>
static void launch_seg(const SegPassDev& p, int threads, size_t lds, hipStream_t s) {
  auto k = k_seg_pass<W, REAL, R>;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  const int64_t blocks = p.xcd_rows > 0 ? 8 * p.xcd_rows * p.n_seg : p.n_rows * p.n_seg;
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(std::min(threads, seg_threads<W, R>())), lds, s, p);
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
