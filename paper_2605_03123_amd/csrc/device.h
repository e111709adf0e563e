// Launchers for the HIP kernels of libffx (kernels.hip).  All launches are
// asynchronous on the given stream; every pointer is device memory.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ffx {
namespace dev {

// One Givens rotation as read by the kernels: local orbital p (relative to the
// window start), cosine c and complex sine (sr, si), and for a real sine the
// shear parameters t = s / (1 + c) and b = -s of x += t y, y += b x, x += t y
// (c >= 0); the f-prefixed fields hold the same values rounded to FP32 (for
// complex64 states).  Built by make_rot.
struct RotDev {
  int p;
  int pad;
  double t, b;
  double c, sr, si;
  float ft, fb;
  float fc, fsr, fsi;
  float fpad;
};
inline RotDev make_rot(int p, double c, double sr, double si) {
  const double t = sr / (1.0 + c), b = -sr;
  return RotDev{p, 0, t, b, c, sr, si, (float)t, (float)b, (float)c, (float)sr, (float)si, 0.0f};
}

// Window class table on the device (see WindowTable in host.h).
struct WinDev {
  const int* tab;
  const int* chunk_m;
  const int* chunk_off;
  const int* cls;
  int n_chunks;
  int n_cls;
  int a, w;
};

// Diagonal function f(I_a, I_b) = A[i_a] + B[i_b] + sum_{p in I_a} V[p * dim_b + i_b].
struct DiagDev {
  const double* A;
  const double* B;
  const double* V;  // may be null (no cross term)
};

// Parameters for building DiagDev tables from occupation vectors:
//   A[i] = lin_a . x + 1/2 x^T Q_a x,  B[i] = lin_b . x + 1/2 x^T Q_b x,
//   V[p][i_b] = (C x_b)[p].  Any matrix pointer may be null (= zero).
struct DiagSpecDev {
  const double* lin_a;
  const double* lin_b;
  const double* Qa;
  const double* Qb;
  const double* C;
};

// Register window of the Givens passes: W = 6 for both precisions (complex64
// also has a W = 7 instantiation, which holds 12 waves instead of 16 and
// measured slower; complex128 at W = 6 fills 143 registers, so 12 waves).
inline int max_window(bool) { return 6; }

// c128 = complex double state, c64 = complex float state.
void win_pass(bool c64, bool real, int spin, void* vec, int64_t dim_a, int64_t dim_b,
              const WinDev& wt, const RotDev* rots, int nrot, const void* phase,
              hipStream_t stream);

// phase[i] = exp(i sum_{p in I_i} delta[p]) in the state's precision.
void string_phase(bool c64, const uint32_t* masks, int64_t n, const double* delta, int norb,
                  void* phase, hipStream_t stream);

void diag_tables(const uint32_t* masks_a, int64_t dim_a, const uint32_t* masks_b, int64_t dim_b,
                 int norb, const DiagSpecDev& spec, double* A, double* B, double* V,
                 hipStream_t stream);

// vec *= exp(i * scale * f)
void diag_phase(bool c64, void* vec, int64_t dim_a, int64_t dim_b, const uint32_t* masks_a,
                int norb, const DiagDev& f, double scale, hipStream_t stream);
// vec *= f
void diag_scale(bool c64, void* vec, int64_t dim_a, int64_t dim_b, const uint32_t* masks_a,
                int norb, const DiagDev& f, hipStream_t stream);
// partials[blk] = sum f |vec|^2 over a block of the state; returns number of partials
int diag_expect(bool c64, const void* vec, int64_t dim_a, int64_t dim_b, const uint32_t* masks_a,
                int norb, const DiagDev& f, double* partials, hipStream_t stream);
int diag_expect_partials(int64_t dim_a, int64_t dim_b);
// out[0] = sum of partials[0..n) in a fixed order
void sum_partials(const double* partials, int n, double* out, hipStream_t stream);
// complex inner product <x|y> in FP64: partials of size 2 * nblocks, out[0..2) = (re, im)
int inner_partials(int64_t n);
void inner(bool c64, const void* x, const void* y, int64_t n, double* partials, double* out,
           hipStream_t stream);

// Chebyshev step: t_prev <- a y + b t_cur + m t_prev; acc += (cr + i ci) t_prev
void cheb_step(bool c64, const void* y, const void* tcur, void* tprev, void* acc, int64_t n, double a,
               double b, double m, double cr, double ci, hipStream_t stream);
// v *= (cr + i ci)
void zscale(bool c64, void* v, int64_t n, double cr, double ci, hipStream_t stream);
// out[0] = sum |x - y|^2 in FP64, fixed order; partials of size inner_partials(n)
void dist2(bool c64, const void* x, const void* y, int64_t n, double* partials, double* out,
           hipStream_t stream);
// State sampling: bs and pre hold sample_blocks(n) doubles each (block sums of
// |gamma|^2 and their inclusive prefix); out[k] = the sampled address for u[k].
int sample_blocks(int64_t n);
int sample_state(bool c64, const void* vec, int64_t n, double* bs, double* pre, const double* u, int64_t n_samples,
                 int64_t* out, hipStream_t stream);
// Dense form of an orbital rotation: C[J, I] = det U[J, I] over the n-electron
// configurations (masks, d of them; U complex norb x norb, device), and the
// complex128 product Y = A B on the FP64 matrix cores (A row-major with leading
// dimension lda; element (k, n) of B at B[k * sbk + n * sbn]; Y row-major, ldy).
void compound_matrix(const uint32_t* masks, int64_t d, int n, int norb, const double* U, void* C, hipStream_t s);
void zgemm_mfma(const void* A, int64_t lda, const void* B, int64_t sbk, int64_t sbn, void* Y, int64_t ldy, int M,
                int N, int K, hipStream_t s);
// The allocation-free sampler's block sums and prefix live in a static device
// array of 2 * kScratchBlocks doubles; sample_scratch returns its address on
// `device` (which must be the current device; taken once per device).
constexpr int64_t kScratchBlocks = (int64_t)1 << 18;
hipError_t sample_scratch(int device, double** ptr);
// Slater-determinant sampling of one spin: Q (N x eta complex, row-major), u
// (n_samples x eta uniforms), masks[k] = the sampled configuration; N, eta <= 32.
void dpp_sample(const double* Q, int N, int eta, const double* u, int64_t n_samples, uint64_t* masks,
                hipStream_t stream);

// optional diagonal term of onebody_rows: w(j, col) = A[j] + B[col] + sum_{p in rmasks[j]} V[p * cols + col]
struct OneBodyDiag {
  const double* A;
  const double* B;
  const double* V;
  const uint32_t* rmasks;
  int norb;
};
// dst[j, :] = sum_{e in [off[j], off[j+1])} coef[e] * src[srow[e], :] (+ w(j, :) src[j, :] when dg.A)
// (+ add[j, :]); dst must not alias src (add may alias dst)
void onebody_rows(bool c64, const void* src, void* dst, const void* add, int64_t rows, int64_t cols,
                  const int64_t* off, const int32_t* srow, const double* coef, const OneBodyDiag& dg,
                  hipStream_t stream);
// y += x
void axpy(bool c64, const void* x, void* y, int64_t n, hipStream_t stream);
// vec[i_a, i_b] = a[i_a] * b[i_b] (a, b complex double)
void outer(bool c64, const double* a, const double* b, void* vec, int64_t dim_a, int64_t dim_b,
           hipStream_t stream);
// dst = src^T (rows x cols -> cols x rows)
void transpose(bool c64, const void* src, void* dst, int64_t rows, int64_t cols,
               hipStream_t stream);

// Transition one-body matrix of the row spin: for every row string I and every
// (p, q) with q in I and (p not in I or p == q), J = I - q + p:
//   part[(p * norb + q) * rows + i] = sign * sum_col conj(lam[J, col]) psi[I, col]
// (zero where (p, q) is not an excitation of I).  Then T[p][q] = sum_i part.
void rdm_rows(bool c64, const void* lam, const void* psi, int64_t rows, int64_t cols,
              const uint32_t* masks_rows, int norb, double* part, hipStream_t stream);
void rdm_reduce(const double* part, int64_t rows, int norb, double* T, hipStream_t stream);
// The same partials for the COLUMN spin through the strings of one electron
// fewer (norb <= 16): T_pq = sum over (n-1)-electron strings K of
// conj(lam[K + p]) psi[K + q] s_p(K) s_q(K), s_x(K) = (-1)^{|K below x|}, as
// 16 x 16 x 4 FP64 matrix-core products whose operands are gathered per lane
// (orbital = lane % 16, string = lane / 16; zero where the orbital is in K).
// The strings K are grouped by their occupation of the top (norb - nlow)
// orbitals; group g's "home" columns [off, off + len) (strings with the same
// top occupation) of lam and psi are staged in LDS, columns outside it are
// read from HBM.  group[4 g ..] = {home_off, home_len, first K, number of K}.
struct RdmMfmaDev {
  const void* lam;
  const void* psi;
  int64_t rows, cols;
  int norb, nlow, ngroups, max_home, max_inter;
  int pad;
  const int* group;
  const uint32_t* inter;
  const int* rank_lo;
  const int* rank_hi;
  double* part;
};
size_t rdm_mfma_lds(bool c64, int max_home, int max_inter);
void rdm_mfma(bool c64, const RdmMfmaDev& d, hipStream_t stream);

// Diagonal-gate gradient reductions (see api): for each row i_a and
//   z = Im(conj(lam) psi), g_0 = 1, g_{1+p} = x_b[p], g_{1+N+p} = x_b[p] x_b[p+1]:
//   rowout[i_a * 2N + k] = sum_{i_b} z * g_k(I_b)
void diag_grad_rows(bool c64, const void* lam, const void* psi, int64_t dim_a, int64_t dim_b,
                    const uint32_t* masks_b, int norb, double* rowout, hipStream_t stream);
// Diagonal-Coulomb matrix gradient rows: rowout[i_a * N^2 + p N + q] =
//   sum_{i_b} Im(conj(lam) psi) (x_a + x_b)_p (x_a + x_b)_q
void dc_grad_rows(bool c64, const void* lam, const void* psi, int64_t dim_a, int64_t dim_b,
                  const uint32_t* masks_a, const uint32_t* masks_b, int norb, double* rowout, hipStream_t stream);
// out[w] = sum_{r < rows} in[r * width + w] in a fixed order (w < width)
void sum_columns(const double* in, int rows, int width, double* out, hipStream_t stream);
// out[p]      (p < N-1) = 2 sum_{i_a} (x_a[p] x_a[p+1] rowout[i_a][0] + rowout[i_a][1+N+p])
// out[N-1+p]  (p < N)   = 2 sum_{i_a} x_a[p] rowout[i_a][1+p]
void diag_grad_combine(const double* rowout, int64_t dim_a, const uint32_t* masks_a, int norb,
                       double* out, hipStream_t stream);

// ---------------------------------------------------------------------------
// segment passes: one block owns one contiguous segment of one row of the
// (possibly transposed) state in LDS and applies a list of stages to it.
// ---------------------------------------------------------------------------
constexpr int kMaxStageRots = 64;  // rotations per Givens stage of a segment pass (one per lane)

enum StageType { ST_GIVENS = 0, ST_PHASE = 1, ST_SCALE = 2, ST_REDUCE = 3 };

// Stage shapes: the window positions, in order, of the rotations of the
// Givens stages that the window schedulers cut from the column-elimination
// network at window width 6 (the full triangle of a 6-orbital window, the
// 3 x 3 parallelogram that sweeps a window across the network, with and
// without its tail, the 4 x 2 parallelogram and its extension to a 14-rotation
// trapezoid that the searched schedules use, the descending diagonal at the
// end, and the forms that appear at small norb).  A stage whose rotation list is one of these runs
// straight-line code with the positions fixed at compile time; any other
// stage runs the generic loop that selects each rotation's position at run
// time.
constexpr int kShapeW = 6;
constexpr int kNumShapes = 10;
constexpr int kShapeMaxLen = 15;
constexpr int kShapeLen[kNumShapes] = {15, 9, 12, 5, 4, 8, 5, 9, 8, 14};
constexpr int kShapeP[kNumShapes][kShapeMaxLen] = {
    {0, 1, 2, 3, 4, 0, 1, 2, 3, 0, 1, 2, 0, 1, 0},
    {2, 3, 4, 1, 2, 3, 0, 1, 2},
    {2, 3, 4, 1, 2, 3, 0, 1, 2, 0, 1, 0},
    {4, 3, 2, 1, 0},
    {3, 2, 1, 0},
    {3, 4, 2, 3, 1, 2, 0, 1},
    {1, 2, 0, 1, 0},
    {3, 4, 2, 3, 1, 2, 0, 1, 0},
    {1, 2, 3, 4, 0, 1, 2, 3},
    {1, 2, 3, 4, 0, 1, 2, 3, 0, 1, 2, 0, 1, 0},
};

// f(row, col) = A[row] + B[col] + sum_{p in row, q in col} C[p * norb + q]
//   ST_PHASE : x *= (-1)^{|row & sign_row|} exp(i (scale (A[row] + cross) + sum_{p in row} drow[p]))
//                   * colf[col]
//              where colf (built per stage) holds the column-only factor
//              (-1)^{|col & sign_col|} exp(i (scale B[col] + sum_{q in col} dcol[q]))
//   ST_SCALE : x *= f
//   ST_REDUCE: accumulate f |x|^2 into the block's partial sum
// ST_GIVENS: the rotations rots[0..nrot) on the window [a, a + W) of the
//   column strings.
struct StageDev {
  int type;
  int a;
  int nrot;
  uint32_t sign_row;
  int shape;  // ST_GIVENS: index into the stage shapes, or -1
  // ST_PHASE: column orbitals whose occupation parity flips the sign (a
  // deferred sign layer of the column spin that needs no column table)
  uint32_t sign_col;
  const RotDev* rots;
  double scale;
  const double* A;
  const double* B;
  const double* C;
  const double* drow;
  const double* colf;  // complex (re, im) per column string
};

// Class tables of one register window inside one segment.  Chunk ch holds 64
// lanes; code[ch * 64 + lane] = (cbase << kCodeMoffBitsDev) | moff for the
// lane's class (-1 for padding), where member k of the class sits at cbase +
// mt_all[moff + k] (moff = mt_off + mt[m * nl1 + l] for m electrons in the
// window and l below it, folded in on the host).  Chunks are listed in order
// of decreasing work; classes with an empty or full window are omitted.
constexpr int kCodeMoffBitsDev = 14;
struct SegWinDev {
  const int* code;
  const int* chunk_m;
  int mt_off;  // start of this window's offsets inside the segment's mt_all
  int n_chunks;
  int nl1;
  int pad;
};

// one segment of a row: [off, off + len) of the column strings, all sharing
// the occupation of the orbitals above the segment window; win[a] holds the
// class tables of the register window [a, a + W), positions relative to off.
struct SegDev {
  int off, len;
  const SegWinDev* win;
  const int* mt_all;  // member offsets of every window, staged into LDS once per block
  int n_mt_all;
  // crossing rotation on (wt - 1, wt), the orbital pair that straddles the
  // segment window: it pairs the strings [cross_lo, cross_lo + cross_cnt) of
  // this segment elementwise with cross_cnt strings from column cross_peer on
  // (same inner order); role 0: this side holds wt - 1 (x' = c x + s y),
  // role 1: it holds wt (y' = c y - conj(s) x)
  int cross_lo, cross_cnt, cross_peer, cross_role;
  int pad;
};

// colf[i] = (-1)^{|mask_i & sign|} exp(i (scale B[i] + sum_{q in mask_i} delta[q]))
void column_factors(const uint32_t* masks, int64_t n, const double* B, double scale, const double* delta,
                    uint32_t sign, double* colf, hipStream_t stream);

enum SegMode { SEG_STORE = 0, SEG_ACCUM = 1, SEG_NONE = 2 };

struct SegPassDev {
  const void* src;
  void* dst;
  int mode;
  int norb;
  int64_t n_rows, row_len;
  const uint32_t* row_masks;
  const uint32_t* col_masks;
  int n_seg;
  int n_stages;
  const SegDev* segs;
  const StageDev* stages;
  double* partials;
  int lds_row_bytes;  // byte offset of the scratch area after the row segment
  int max_mt;         // ints reserved in LDS for the member offsets of all windows
  // when set, the crossing rotation (cross_c, cross_sr + i cross_si) is applied
  // as the segment is loaded, reading the partner strings from src (which the
  // pass must not overwrite: src != dst)
  int cross;
  double cross_c, cross_sr, cross_si;
  // gather: src holds the state in the other layout (element (r, c) of this
  // pass at src[c * n_rows + r]), so the pass also transposes (it must not
  // write src).
  int gather;
  // scatter: dst receives the state in the other layout (element (r, c) of this
  // pass at dst[c * n_rows + r]), so the pass also transposes (dst != src).
  int scatter;
  // xcd_rows > 0: blocks take rows per XCD: block b works on XCD b % 8, on row
  // (b % 8) * xcd_rows + (b / 8) / n_seg, segment (b / 8) % n_seg, so that the
  // blocks of one XCD gather neighbouring columns of the same cache lines, and
  // the segments of one row (whose crossing partners overlap) share an L2
  int64_t xcd_rows;
};

// Segment passes on row planes (complex128 row segments of at most
// seg_pass_plane_max_len(threads) amplitudes, real Givens rotations only): the
// real and imaginary parts are rotated in turn, one in LDS (len * 8 bytes of
// row area in `lds`) and the other in registers.
// W in 4..6 (6 where rows are split into several segments); threads 512 or 768.
int seg_pass_plane_max_len(int threads);
void seg_pass_planes(int W, int threads, const SegPassDev& p, size_t lds, hipStream_t stream);


// LDS needed by a segment pass whose longest segment holds max_len amplitudes
// ---------------------------------------------------------------------------
// batched persistent launch: many independent sectors, each running a list of
// passes; one kernel pulls tasks (blocks of rows or columns of one instance's
// state) from a global queue in pass-level order, and a task starts only when
// every task of its instance's earlier passes has finished.
// ---------------------------------------------------------------------------
enum BatchKind { BK_TABLES = 0, BK_OUTER = 1, BK_SEG = 2, BK_INNER = 3, BK_RDM = 4, BK_DGRAD = 5, BK_SUM = 6 };

// one sector type (norb, n_alpha, n_beta) shared by instances
struct BTypeDev {
  int norb;
  int n[2];
  int pad;
  int64_t dim[2];
  const uint32_t* masks[2];
  // per column spin cs: tasks of the layout whose columns are spin cs hold
  // rows_per_task[cs] rows; window tables replicated over those rows
  int rows_per_task[2];
  const SegWinDev* win[2];
  const int* mt_all[2];
  int n_mt_all[2];
  // per string spin s, for the transition one-body matrices: the strings K of
  // n_s - 1 electrons, nk[s] of them, and for each K and orbital o < 16:
  // kt[s][16 K + o] = 2 rank(K + o) + parity(K below o) if o < norb and o is
  // not in K, else -1
  const int* kt[2];
  int nk[2];
};

// one table of a TABLES pass: a diagonal function's per-string tables (A over
// alpha strings, B over beta strings), or one phase stage's column factors
struct BTableDev {
  int kind;  // 0: diagonal tables, 1: column factors
  int spin;  // column factors: the strings' spin
  DiagSpecDev spec;
  double* A;
  double* B;
  const double* cB;
  double scale;
  const double* delta;
  uint32_t sign;
  int pad;
  double* out;
};

struct BPassDev {
  int kind;
  int type;      // index into the sector types
  int inst;      // instance (dependency counter)
  int layout;    // 0: rows are alpha strings, 1: rows are beta strings (columns of the state)
  int mode;      // SEG: SegMode
  int real;      // SEG: all rotations real
  int n_stages;
  int n_tasks;
  int half;      // SEG: tasks >= half use (src2, dst2) (two states, same stages); else n_tasks
  int need;      // finished tasks of this instance required before any task of this pass
  int width;     // SUM: doubles per partial vector; others: doubles of partials per task
  int n_sum;     // SUM: number of partial vectors
  int64_t first;  // queue index of the first task
  const StageDev* stages;
  const void* src;
  void* dst;
  const void* src2;
  void* dst2;
  double* partials;
  double* out;
  const BTableDev* tables;
  const double* oa;  // OUTER: complex per alpha string
  const double* ob;  // OUTER: complex per beta string
};

struct BatchDev {
  const BTypeDev* types;
  const BPassDev* passes;
  int n_passes;
  int pad;
  int64_t n_tasks;
  unsigned int* next;     // queue counter
  unsigned int* done;     // per instance: finished tasks
  unsigned int* abort;    // set when a wait exceeds its bound
  int lds_row_bytes;      // LDS bytes reserved for the rows of one task
  int max_mt;             // ints reserved for member-offset tables
  int wq_rows;            // rows reserved for the cross weights and row factors (the most rows of a task)
  int pad2;
};

// LDS bytes of the batched kernel and its launch.  blocks: resident blocks to start.
size_t batch_lds(bool c64, int lds_row_bytes, int max_mt, int wq_rows);
// LDS bytes of a launch that runs tasks of one kind only
size_t batch_lds_for(int kind, int lds_row_bytes, int max_mt, int wq_rows);
int batch_blocks_per_cu(bool c64, int threads, size_t lds);
void batch_launch(bool c64, const BatchDev& b, int blocks, int threads, size_t lds, hipStream_t s);
// level-synchronous form: the tasks of passes [p0, p1) (one level), one block each
// passes [p0, p1) of one level, all of kind `kind`, one block per task
void batch_launch_kind(bool c64, int kind, const BatchDev& b, int p0, int p1, int64_t tasks, size_t lds,
                       hipStream_t s);

// single cooperative launch over all levels (grid barrier between levels); blocks must not exceed
// batch_coop_blocks_per_cu(...) times the compute units (the launch fails otherwise)
int batch_coop_blocks_per_cu(bool c64, size_t lds);
// level_ctr: n_levels task counters, zero at launch
hipError_t batch_launch_coop(bool c64, const BatchDev& b, const int* level_start, int n_levels,
                             unsigned int* level_ctr, int blocks, size_t lds, hipStream_t s);

size_t seg_pass_lds(bool c64, int max_len, int max_mt);
// block size a segment pass launches with for a requested size (the kernel's
// register budget caps it)
int seg_pass_threads(bool c64, int W, int requested);
// blocks = n_rows * n_seg; partials (if any stage reduces) get one entry per block
void seg_pass(bool c64, bool real, int W, const SegPassDev& p, int block_threads, size_t lds_bytes,
              hipStream_t stream);
// in-place transpose of a square n x n state
void transpose_square(bool c64, void* vec, int64_t n, hipStream_t stream);

}  // namespace dev
}  // namespace ffx
