// Internal: the plan object, the pinned parameter-upload ring and the gate
// program compiler of libffx.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "device.h"
#include "ffx.h"
#include "host.h"

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw ffx::Error(FFX_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));     \
  } while (0)

namespace ffx {
void check_launch();
}

struct ffx_plan_s {
  int norb = 0;
  int n[2] = {0, 0};
  bool c64 = false;
  int device = 0;
  int64_t dim[2] = {0, 0};
  std::vector<uint64_t> str[2];
  uint32_t* d_masks[2] = {nullptr, nullptr};
  int W = 2;                          // register window of whole-spin window passes
  std::vector<ffx::dev::WinDev> win[2];
  // segment passes, per column spin
  struct SegSet {
    int wt = 0;        // segments share the occupation of orbitals >= wt
    int Wseg = 0;      // register window inside segment passes (windows within [0, wt))
    int max_len = 0;
    int max_mt = 0;
    int n_seg = 0;
    size_t lds = 0;
    int threads = 256;
    bool cross = false;  // rotations on (wt - 1, wt) can be applied at segment load
    ffx::dev::SegDev* d_segs = nullptr;
  } seg[2];
  // whole rows as two planes (complex128 rows that exceed LDS but whose real
  // parts fit): one segment per row, for visits whose rotations are all real;
  // n_seg = 0 where unavailable
  SegSet plane[2];
  // parameter upload ring
  static constexpr int kSlots = 4;
  size_t slot_bytes = 0;
  char* h_ring = nullptr;
  char* d_ring = nullptr;
  hipEvent_t ev[kSlots] = {};
  int next_slot = 0;
  // scratch
  void* phase_tab[2] = {nullptr, nullptr};
  double* dA = nullptr;
  double* dB = nullptr;
  double* dV = nullptr;
  double* partials = nullptr;
  int n_partials = 0;
  double* results = nullptr;  // results_cap doubles (kResults at creation, grown by results_for)
  size_t results_cap = 0;
  double* rowout = nullptr;
  void* state_tmp = nullptr;   // one state, allocated on first need
  double* arena = nullptr;     // per-program diagonal tables
  size_t arena_doubles = 0;
  std::vector<void*> allocs;
  static constexpr int kResults = 1 << 16;
  // diagnostics: event pairs around the dominant launches
  struct Timed {
    hipEvent_t a, b;
    int kind;  // 0 window pass, 1 segment pass, 2 segment pass on row planes
    int spin;
    double alg_bytes;
    double valu_slots;
  };
  bool timing = false;
  std::vector<Timed> timed;
  std::vector<hipEvent_t> ev_pool;

  hipEvent_t take_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
  void recycle_timed() {
    for (auto& t : timed) {
      ev_pool.push_back(t.a);
      ev_pool.push_back(t.b);
    }
    timed.clear();
  }

  size_t elem() const { return c64 ? 8 : 16; }
  int64_t elems() const { return dim[0] * dim[1]; }
  size_t state_bytes() const { return (size_t)elems() * elem(); }

  void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (ffx::fault_hit("alloc") || hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess || !p)
      throw ffx::Error(FFX_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    allocs.push_back(p);
    return p;
  }
  void* tmp_state() {
    if (!state_tmp) state_tmp = dalloc(state_bytes());
    return state_tmp;
  }
  // per-program diagonal tables; every program of a call starts at offset 0
  // (programs run one after another on the stream).  Growing frees the old
  // arena, so a driver that compiles several programs before running them must
  // stay within the initial size (kArenaSlots states' worth of string tables).
  // colex rank of a mask by bytes (norb <= 16), built on first use:
  // rank = rank_lo[m & 255] + rank_hi[(m >> 8) * 17 + popcount(m & 255)]
  int* rank_lo = nullptr;
  int* rank_hi = nullptr;
  bool rdm_pairs = false;  // transition one-body matrices from row pairs at any size
  // standalone orbital rotations of complex128 sectors with at most this many
  // configurations per spin take the dense form on the matrix cores (measured
  // faster than the Givens sweeps at 70 configurations, even at 252, slower above)
  int64_t dense_max_dim = 128;
  void* dense_ws = nullptr;  // its compound matrices and intermediate, allocated on first use
  // per column spin: the (n-1)-electron strings for the matrix-core transition
  // one-body kernel, grouped by their top occupation, built on first use
  struct RdmStrings {
    bool ready = false;
    int nlow = 0, ngroups = 0, max_home = 0, max_inter = 0;
    int* group = nullptr;
    uint32_t* inter = nullptr;
  } rdm_k[2];
  // when set, compile_program takes its table arena from this hook instead
  double* (*arena_hook)(void* ctx, size_t doubles) = nullptr;
  void* arena_ctx = nullptr;
  int max_stage_rots = ffx::dev::kMaxStageRots;  // Givens rotations per stage (fusion depth)
  static constexpr int kArenaSlots = 64;
  // the device result block, grown to at least `doubles`.  The new block is
  // allocated before the old one is released (after waiting for the device,
  // since earlier work on any stream may still use it), so a failed
  // allocation leaves the plan with its old block.
  double* results_for(size_t doubles, hipStream_t s) {
    if (doubles > results_cap) {
      double* grown = (double*)dalloc(doubles * sizeof(double));
      release_block(results, s);
      results = grown;
      results_cap = doubles;
    }
    return results;
  }
  double* arena_for(size_t doubles, hipStream_t s) {
    if (doubles > arena_doubles) {
      double* grown = (double*)dalloc(doubles * sizeof(double));
      release_block(arena, s);
      arena = grown;
      arena_doubles = doubles;
    }
    return arena;
  }
  void release_block(double* p, hipStream_t s) {
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipDeviceSynchronize());
    auto it = std::find(allocs.begin(), allocs.end(), (void*)p);
    if (it != allocs.end()) allocs.erase(it);
    if (p) (void)hipFree(p);
  }

  ~ffx_plan_s() {
    recycle_timed();
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : allocs) (void)hipFree(p);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (h_ring) (void)hipHostFree(h_ring);
  }
};

namespace ffx {

// One slot of the pinned upload ring: small per-call data is packed here,
// copied to the device once, and read by the kernels of that call.
struct Upload {
  ffx_plan_s* P;
  int slot;
  char* h;
  char* d;
  size_t cap;
  size_t off = 0;
  hipStream_t s;

  // over caller buffers (no slot event); h == nullptr only measures the size
  Upload(char* host, char* dev, size_t capacity, hipStream_t stream)
      : P(nullptr), slot(-1), h(host), d(dev), cap(capacity), s(stream) {}
  Upload(ffx_plan_s* plan, hipStream_t stream) : P(plan), s(stream) {
    slot = P->next_slot;
    P->next_slot = (P->next_slot + 1) % ffx_plan_s::kSlots;
    HIPCHK(hipEventSynchronize(P->ev[slot]));  // previous user of the slot is done
    h = P->h_ring + (size_t)slot * P->slot_bytes;
    d = P->d_ring + (size_t)slot * P->slot_bytes;
    cap = P->slot_bytes;
  }
  template <class T>
  const T* put(const T* src, size_t count) {
    off = (off + 15) & ~(size_t)15;
    size_t bytes = count * sizeof(T);
    if (off + bytes > cap) throw Error(FFX_EUNSUPPORTED, "parameter block exceeds the upload slot");
    if (bytes && h) std::memcpy(h + off, src, bytes);
    const T* r = (const T*)(d + off);
    off += bytes;
    return r;
  }
  void commit() {
    if (off && h) HIPCHK(hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, s));
  }
  ~Upload() {
    if (P) (void)hipEventRecord(P->ev[slot], s);
  }
};

// ---------------------------------------------------------------------------
// gate programs
// ---------------------------------------------------------------------------
// A diagonal function f(I_a, I_b) = lin_a.x_a + lin_b.x_b + 1/2 x_a Qa x_a
// + 1/2 x_b Qb x_b + x_a C x_b (host arrays, any may be null).
struct DiagSpec {
  const double* lin_a = nullptr;
  const double* lin_b = nullptr;
  const double* Qa = nullptr;
  const double* Qb = nullptr;
  const double* C = nullptr;
};

struct ProgOp {
  enum Kind { ROT, PHASE, SCALE, REDUCE } kind;
  const Decomposition* part[2] = {nullptr, nullptr};  // ROT: alpha and beta parts
  int diag = -1;                                      // PHASE / SCALE / REDUCE
  double scale = 0.0;                                 // PHASE: x *= exp(i scale f)
  double* out = nullptr;                              // REDUCE: device result slot
};

struct Program {
  std::vector<DiagSpec> diags;
  std::vector<ProgOp> ops;
  int add_diag(const DiagSpec& d) {
    diags.push_back(d);
    return (int)diags.size() - 1;
  }
  void rot(const Decomposition* a, const Decomposition* b) {
    ProgOp o{ProgOp::ROT};
    o.part[0] = a;
    o.part[1] = b;
    ops.push_back(o);
  }
  void phase(int diag, double scale) {
    ProgOp o{ProgOp::PHASE};
    o.diag = diag;
    o.scale = scale;
    ops.push_back(o);
  }
  void scale(int diag) {
    ProgOp o{ProgOp::SCALE};
    o.diag = diag;
    ops.push_back(o);
  }
  void reduce(int diag, double* out) {
    ProgOp o{ProgOp::REDUCE};
    o.diag = diag;
    o.out = out;
    ops.push_back(o);
  }
};

enum FinalMode { FINAL_STORE = 0, FINAL_ACCUM = 1, FINAL_NONE = 2 };

struct Launch {
  enum Kind { SEG, WIN, TRANSPOSE, SUM } kind;
  int layout = 0;  // 0: rows alpha / columns beta; 1: rows beta / columns alpha
  bool real = true;
  // SEG
  const dev::StageDev* stages = nullptr;
  int n_stages = 0;
  bool reduce = false;
  double* reduce_out = nullptr;
  double valu_slots = 0;
  double rot_sides = 0;
  // a rotation on the pair straddling the segment window, applied at load
  bool cross = false;
  // rows gathered from the other layout (replaces a transpose before the pass)
  bool gather = false;
  // rows stored as columns of the other layout (replaces a transpose after the pass)
  bool scatter = false;
  // the row held as two planes (the plan's plane set of the column spin)
  bool planes = false;
  dev::RotDev cross_rot{};
  // WIN
  int a = 0;
  const dev::RotDev* rots = nullptr;
  int nrot = 0;
};

struct TableBuild {
  dev::DiagSpecDev spec;
  double* A;  // per alpha string
  double* B;  // per beta string
};

struct ColfBuild {
  int spin;          // column spin: its configuration masks
  const double* B;   // per-string table (nullable)
  double scale;
  const double* delta;
  uint32_t sign;
  double* out;       // complex per string
};

struct Compiled {
  std::vector<TableBuild> tables;
  std::vector<ColfBuild> colfs;
  std::vector<Launch> launches;
  int final_mode = FINAL_STORE;
};

// Writes the program's parameters into the upload (before commit) and returns
// the launch list; diagonal tables are built on the device at execution.
Compiled compile_program(ffx_plan_s& P, Upload& up, const Program& prog, int final_mode, hipStream_t s);
// src -> work (src may equal work); FINAL_ACCUM adds the result into accum.
void execute_program(ffx_plan_s& P, const Compiled& c, const void* src, void* work, void* accum,
                     hipStream_t s);

}  // namespace ffx
