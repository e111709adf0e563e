// Batched LUCJ energy + adjoint gradient (include/ffx.h, ffx_batch_*): the
// gate programs of every instance are compiled against one plan per sector
// type, turned into passes of tasks (blocks of rows or columns), ordered pass
// level by pass level across instances, and run by one cooperative launch
// with a grid barrier between levels, or by one launch per level (batched.hip).  The host then applies each instance's gradient chain rule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <memory>
#include <numeric>
#include <string>
#include <tuple>
#include <exception>
#include <thread>
#include <vector>

#include "device.h"
#include "drivers.h"
#include "ffx.h"
#include "host.h"
#include "plan.h"

using namespace ffx;

struct ffx_batch_s {
  bool c64 = false;
  int device = 0;
  int n_inst = 0;
  std::vector<int> inst_type;
  std::vector<std::tuple<int, int, int>> type_key;  // (norb, n_a, n_b)
  std::vector<ffx_plan> plans;
  std::vector<dev::BTypeDev> htypes;
  dev::BTypeDev* d_types = nullptr;
  std::vector<void*> table_allocs;  // replicated class tables (rebuilt by the tuner)
  int target_elems = 4096;
  int stage_rots = dev::kMaxStageRots;
  int lds_row_bytes = 0;
  int max_mt = 0;
  int wq_rows = 1;  // the most rows of a segment task (cross weights and row factors in LDS)
  size_t lds = 0;
  int blocks = 0;
  // One persistent launch for the whole batch (task queue with per-instance
  // dependency counters) instead of one launch per pass level.  Off: its last
  // run on the GPU did not complete and the cause is not established.
  bool persistent = false;
  // One cooperative launch that walks the pass levels with a grid barrier
  // between them (ffx_batch_single_launch(batch, 1)); by default one launch per
  // pass kind of each level, each with its kind's own registers and LDS (about
  // a quarter faster on the 256-sector workload).
  bool single_launch = false;
  // timing of the last call
  double last_device_ms = 0, last_call_ms = 0;
  int last_launches = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // per-call buffers, grown on demand
  char* h_up = nullptr;
  char* d_up = nullptr;
  size_t up_cap = 0;
  double* arena = nullptr;
  size_t arena_cap = 0;
  size_t arena_used = 0;
  double* scratch = nullptr;  // partials and results
  size_t scratch_cap = 0;
  unsigned* counters = nullptr;
  size_t counters_cap = 0;

  ~ffx_batch_s() {
    free_tables();
    if (d_types) (void)hipFree(d_types);
    if (h_up) (void)hipHostFree(h_up);
    if (d_up) (void)hipFree(d_up);
    if (arena) (void)hipFree(arena);
    if (scratch) (void)hipFree(scratch);
    if (counters) (void)hipFree(counters);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    for (ffx_plan p : plans) ffx_plan_destroy(p);
  }
  void free_tables() {
    for (void* p : table_allocs) (void)hipFree(p);
    table_allocs.clear();
  }
  void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (fault_hit("alloc") || hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess || !p)
      throw Error(FFX_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    return p;
  }
  template <class T>
  T* upload_table(const std::vector<T>& v) {
    T* d = (T*)dalloc(std::max<size_t>(v.size(), 1) * sizeof(T));
    table_allocs.push_back(d);
    if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
  }
  size_t elem() const { return c64 ? 8 : 16; }
};

namespace {

int kernel_window(bool c64) { return dev::max_window(c64); }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// fn(i) for i in [0, n) on up to 16 host threads (thread w takes i = w, w + nt,
// ...); the first exception thrown is rethrown after all threads have joined
template <class F>
void parallel_for(int n, F fn) {
  const int nt = std::max(1, std::min<int>({n, 16, (int)std::thread::hardware_concurrency()}));
  std::vector<std::thread> th;
  std::vector<std::exception_ptr> err(nt);
  for (int w = 0; w < nt; ++w)
    th.emplace_back([&, w] {
      try {
        for (int i = w; i < n; i += nt) fn(i);
      } catch (...) {
        err[w] = std::current_exception();
      }
    });
  for (auto& t : th) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

// rows of a transition-matrix task: half those of a segment task (two states in LDS)
int64_t rdm_rows(int seg_rows) { return seg_rows > 1 ? seg_rows / 2 : 1; }

// class tables of the batched kernel for the current target: rows per task
// per layout, replicated window tables, LDS size and resident blocks
void build_tables(ffx_batch_s& b) {
  b.free_tables();
  b.lds_row_bytes = 16;
  b.max_mt = 0;
  b.wq_rows = 1;
  for (size_t ti = 0; ti < b.plans.size(); ++ti) {
    const ffx_plan_s& P = *b.plans[ti];
    dev::BTypeDev& t = b.htypes[ti];
    t.norb = P.norb;
    t.n[0] = P.n[0];
    t.n[1] = P.n[1];
    t.dim[0] = P.dim[0];
    t.dim[1] = P.dim[1];
    t.masks[0] = P.d_masks[0];
    t.masks[1] = P.d_masks[1];
    for (int cs = 0; cs < 2; ++cs) {
      const auto& ss = P.seg[cs];
      const int64_t len = P.dim[cs], nrows = P.dim[1 - cs];
      int R = (int)std::max<int64_t>(1, b.target_elems / std::max<int64_t>(len, 1));
      R = (int)std::min<int64_t>({(int64_t)R, (int64_t)64, std::max<int64_t>(nrows, 1)});
      t.rows_per_task[cs] = R;
      b.wq_rows = std::max(b.wq_rows, R);
      std::vector<dev::SegWinDev> wins;
      std::vector<int> mt_all;
      for (int a = 0; ss.Wseg >= 2 && a + ss.Wseg <= ss.wt; ++a) {
        SegWindowTable one = build_seg_window(P.str[cs], ss.wt, a, ss.Wseg);
        SegWindowTable rep = replicate_seg_window(one, ss.Wseg, R, (int)len);
        dev::SegWinDev wd{};
        while (mt_all.size() % 4) mt_all.push_back(0);
        wd.mt_off = (int)mt_all.size();
        wd.code = b.upload_table(pack_class_codes(rep, wd.mt_off));
        wd.chunk_m = b.upload_table(rep.chunk_m);
        wd.n_chunks = (int)rep.chunk_m.size();
        wd.nl1 = rep.nl1;
        mt_all.insert(mt_all.end(), rep.mt.begin(), rep.mt.end());
        wins.push_back(wd);
      }
      // the strings of one electron fewer and their one-orbital completions
      {
        const int N = P.norb, n = P.n[cs];
        std::map<uint64_t, int> addr;
        for (size_t k = 0; k < P.str[cs].size(); ++k) addr[P.str[cs][k]] = (int)k;
        std::vector<int> kt;
        int nk = 0;
        if (n >= 1)
          for (uint32_t K = 0; K < (1u << N); ++K) {
            if (__builtin_popcount(K) != n - 1) continue;
            ++nk;
            for (int o = 0; o < 16; ++o) {
              if (o >= N || ((K >> o) & 1u)) {
                kt.push_back(-1);
                continue;
              }
              const int odd = __builtin_popcount(K & ((1u << o) - 1u)) & 1;
              kt.push_back(2 * addr.at((uint64_t)(K | (1u << o))) + odd);
            }
          }
        if (kt.empty()) kt.push_back(-1);
        t.kt[cs] = b.upload_table(kt);
        t.nk[cs] = nk;
      }
      t.win[cs] = b.upload_table(wins);
      while (mt_all.size() % 4) mt_all.push_back(0);  // staged as int4 words
      t.mt_all[cs] = b.upload_table(mt_all);
      t.n_mt_all[cs] = (int)mt_all.size();
      b.max_mt = std::max(b.max_mt, (int)mt_all.size());
      // a segment task holds R rows; a transition-matrix task holds rdm_rows(R) rows of two states
      const size_t rows_held = std::max<size_t>((size_t)R, 2 * (size_t)rdm_rows(R));
      const size_t rb = (rows_held * (size_t)len * b.elem() + 15) & ~(size_t)15;
      b.lds_row_bytes = std::max<int>(b.lds_row_bytes, (int)rb);
    }
  }
  b.lds = dev::batch_lds(b.c64, b.lds_row_bytes, b.max_mt, b.wq_rows);
  if (b.lds > 160 * 1024 - 256) throw Error(FFX_EUNSUPPORTED, "batched task rows exceed LDS; lower the target");
  if (!b.d_types) b.d_types = (dev::BTypeDev*)b.dalloc(b.htypes.size() * sizeof(dev::BTypeDev));
  HIPCHK(hipMemcpy(b.d_types, b.htypes.data(), b.htypes.size() * sizeof(dev::BTypeDev), hipMemcpyHostToDevice));
  int per_cu = dev::batch_blocks_per_cu(b.c64, 256, b.lds);
  if (per_cu < 1) throw Error(FFX_EUNSUPPORTED, "batched kernel does not fit on a compute unit");
  int cus = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b.device));
  b.blocks = per_cu * cus;
}

size_t state_bytes(const ffx_batch_s& b, int i) {
  const ffx_plan_s& P = *b.plans[b.inst_type[i]];
  return ((size_t)P.state_bytes() + 255) / 256 * 256;
}

double* arena_hook(void* ctx, size_t doubles) {
  ffx_batch_s& b = *(ffx_batch_s*)ctx;
  double* p = b.arena ? b.arena + b.arena_used : (double*)nullptr;
  b.arena_used += (doubles + 31) & ~(size_t)31;
  return p ? p : (double*)(uintptr_t)(256 + 8 * b.arena_used);  // measuring: any distinct address
}



// the passes of one instance, in order, with their local dependency counts
struct InstPasses {
  std::vector<dev::BPassDev> p;
  int64_t tasks = 0;
  void add(dev::BPassDev x) {
    x.need = (int)tasks;
    if (x.half == 0) x.half = x.n_tasks;
    tasks += x.n_tasks;
    p.push_back(x);
  }
};

struct InstBuild {
  std::unique_ptr<LUCJGrad> G;
  Compiled fwd;
  std::vector<Compiled> terms, urot, udiag;
  const double* sa = nullptr;
  const double* sb = nullptr;
  size_t res_off = 0;    // doubles into the result block
  size_t part_off = 0;   // doubles into the partials block
  size_t part_need = 0;
};

// one call: compile, build passes, launch, assemble
void run_batch(ffx_batch_s& b, const ffx_lucj* ops, const ffx_df_ham* hams, double* energies, double* grads,
               void* workspace, hipStream_t s, float* kernel_ms, std::vector<int64_t>* queue = nullptr) {
  const int n = b.n_inst;
  std::vector<InstBuild> ib(n);
  // the per-instance decompositions and gate programs are independent: built
  // on several host threads (plans are only read)
  parallel_for(n, [&](int i) { ib[i].G = build_lucj_grad(*b.plans[b.inst_type[i]], &ops[i], &hams[i]); });
  // compile every program twice: once to measure the upload and the table
  // arena, once into the allocated buffers
  auto compile_all = [&](Upload& up) {
    b.arena_used = 0;
    for (int i = 0; i < n; ++i) {
      ffx_plan_s& P = *b.plans[b.inst_type[i]];
      P.arena_hook = arena_hook;
      P.arena_ctx = &b;
      P.max_stage_rots = b.stage_rots;
      InstBuild& x = ib[i];
      LUCJGrad& G = *x.G;
      x.sa = up.put((const double*)G.g.a.data(), 2 * G.g.a.size());
      x.sb = up.put((const double*)G.g.b.data(), 2 * G.g.b.size());
      x.fwd = compile_program(P, up, G.fwd, FINAL_STORE, s);
      x.terms.clear();
      x.urot.clear();
      x.udiag.clear();
      for (int t = 0; t <= G.df.L; ++t)
        x.terms.push_back(compile_program(P, up, G.terms[t], t == 0 ? FINAL_STORE : FINAL_ACCUM, s));
      for (int k = 0; k < G.L.R; ++k) {
        x.urot.push_back(compile_program(P, up, G.undo_rot[k], FINAL_STORE, s));
        x.udiag.push_back(compile_program(P, up, G.undo_diag[k], FINAL_STORE, s));
      }
      P.arena_hook = nullptr;
      P.arena_ctx = nullptr;
      P.max_stage_rots = dev::kMaxStageRots;
    }
  };
  struct HookReset {
    ffx_batch_s& b;
    ~HookReset() {
      for (ffx_plan p : b.plans) {
        p->arena_hook = nullptr;
        p->arena_ctx = nullptr;
        p->max_stage_rots = dev::kMaxStageRots;
      }
    }
  } hook_reset{b};
  size_t up_need = 0, arena_need = 0;
  {
    Upload m(nullptr, (char*)(uintptr_t)256, (size_t)1 << 40, s);
    // measured with no arena (the hook hands out stand-in addresses); the
    // arena comes back also when the measuring compile throws
    struct KeepArena {
      double*& slot;
      double* saved;
      ~KeepArena() { slot = saved; }
    } keep{b.arena, b.arena};
    b.arena = nullptr;
    compile_all(m);
    up_need = m.off;
    arena_need = b.arena_used;
  }
  // per instance: results and partial sums
  size_t res_total = 0, part_total = 0;
  for (int i = 0; i < n; ++i) {
    const ffx_plan_s& P = *b.plans[b.inst_type[i]];
    const dev::BTypeDev& t = b.htypes[b.inst_type[i]];
    const int N = P.norb, NN = N * N, R = ib[i].G->L.R;
    const int64_t tr0 = ceil_div(P.dim[0], t.rows_per_task[1]);  // layout 0 tasks
    const int64_t tr1 = ceil_div(P.dim[1], t.rows_per_task[0]);  // layout 1 tasks
    const int64_t td0 = ceil_div(P.dim[0], rdm_rows(t.rows_per_task[1]));  // transition-matrix tasks
    const int64_t td1 = ceil_div(P.dim[1], rdm_rows(t.rows_per_task[0]));
    ib[i].res_off = res_total;
    res_total += 2 + (size_t)R * (4 * NN + 2 * N - 1);
    ib[i].part_need = (size_t)std::max<int64_t>({(td0 + td1) * 2 * NN, tr0 * (2 * N - 1), tr0 * 2});
    ib[i].part_off = part_total;
    part_total += ib[i].part_need;
  }
  // passes are uploaded after the programs' data
  std::vector<InstPasses> ip(n);
  std::vector<std::vector<dev::BTableDev>> tabs(n);
  // build passes with device addresses (needs workspace, scratch)
  char* ws = (char*)workspace;
  std::vector<size_t> ws_off(n);
  {
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
      ws_off[i] = off;
      off += 3 * state_bytes(b, i);
    }
  }
  if (b.scratch_cap < res_total + part_total) {
    if (b.scratch) (void)hipFree(b.scratch);
    b.scratch = nullptr;
    b.scratch_cap = 0;
    b.scratch = (double*)b.dalloc((res_total + part_total) * sizeof(double));
    b.scratch_cap = res_total + part_total;
  }
  double* results = b.scratch;
  double* partials = b.scratch + res_total;
  if (b.arena_cap < arena_need) {
    if (b.arena) (void)hipFree(b.arena);
    b.arena = nullptr;
    b.arena_cap = 0;
    b.arena = (double*)b.dalloc(std::max<size_t>(arena_need, 1) * sizeof(double));
    b.arena_cap = arena_need;
  }
  // the pass list is appended to the upload: bound its size from the programs
  size_t n_pass_bound = 0, n_table_bound = 0;
  for (int i = 0; i < n; ++i) {
    auto count = [&](const Compiled& c) {
      n_pass_bound += c.launches.size();
      n_table_bound += c.tables.size() + c.colfs.size();
    };
    count(ib[i].fwd);
    for (auto& c : ib[i].terms) count(c);
    for (auto& c : ib[i].urot) count(c);
    for (auto& c : ib[i].udiag) count(c);
    n_pass_bound += 8 + 10 * (size_t)ib[i].G->L.R;
  }
  const size_t up_total = up_need + 64 + (n_pass_bound + 4) * (sizeof(dev::BPassDev) + sizeof(int)) +
                          (n_table_bound + 4) * sizeof(dev::BTableDev) + 4096;
  if (b.up_cap < up_total) {
    if (b.h_up) (void)hipHostFree(b.h_up);
    if (b.d_up) (void)hipFree(b.d_up);
    b.h_up = nullptr;
    b.d_up = nullptr;
    b.up_cap = 0;
    if (fault_hit("alloc") || hipHostMalloc((void**)&b.h_up, up_total, hipHostMallocDefault) != hipSuccess)
      throw Error(FFX_ENOMEM, "pinned host allocation of the upload buffer failed");
    b.d_up = (char*)b.dalloc(up_total);
    b.up_cap = up_total;
  }
  Upload up(b.h_up, b.d_up, b.up_cap, s);
  compile_all(up);
  if (up.off != up_need || b.arena_used != arena_need)
    throw Error(FFX_EDEVICE, "batched program compilation is not reproducible");

  // ---- passes ---------------------------------------------------------
  for (int i = 0; i < n; ++i) {
    const int ty = b.inst_type[i];
    const ffx_plan_s& P = *b.plans[ty];
    const dev::BTypeDev& t = b.htypes[ty];
    InstBuild& x = ib[i];
    const LUCJGrad& G = *x.G;
    const int N = P.norb, NN = N * N, R = G.L.R;
    const int64_t tr0 = ceil_div(P.dim[0], t.rows_per_task[1]);
    const int64_t tr1 = ceil_div(P.dim[1], t.rows_per_task[0]);
    const int64_t td0 = ceil_div(P.dim[0], rdm_rows(t.rows_per_task[1]));
    const int64_t td1 = ceil_div(P.dim[1], rdm_rows(t.rows_per_task[0]));
    void* psi = ws + ws_off[i];
    void* lam = ws + ws_off[i] + state_bytes(b, i);
    void* tmp = ws + ws_off[i] + 2 * state_bytes(b, i);
    double* res = results + x.res_off;
    double* part = partials + x.part_off;
    InstPasses& Q = ip[i];
    auto base = [&](int kind) {
      dev::BPassDev p{};
      p.kind = kind;
      p.type = ty;
      p.inst = i;
      return p;
    };
    // tables of every program: the per-string diagonal tables first, then (a
    // pass later, since they read those tables) the column phase factors
    std::vector<dev::BTableDev>& tb = tabs[i];
    std::vector<dev::BTableDev> tc;
    auto add_tables = [&](const Compiled& c) {
      for (const TableBuild& x2 : c.tables) {
        dev::BTableDev e{};
        e.kind = 0;
        e.spec = x2.spec;
        e.A = x2.A;
        e.B = x2.B;
        tb.push_back(e);
      }
      for (const ColfBuild& x2 : c.colfs) {
        dev::BTableDev e{};
        e.kind = 1;
        e.spin = x2.spin;
        e.cB = x2.B;
        e.scale = x2.scale;
        e.delta = x2.delta;
        e.sign = x2.sign;
        e.out = x2.out;
        tc.push_back(e);
      }
    };
    add_tables(x.fwd);
    for (auto& c : x.terms) add_tables(c);
    for (auto& c : x.urot) add_tables(c);
    for (auto& c : x.udiag) add_tables(c);
    for (const auto* list : {&tb, &tc}) {
      if (list->empty()) continue;
      dev::BPassDev p = base(dev::BK_TABLES);
      p.n_tasks = (int)list->size();
      p.tables = up.put(list->data(), list->size());
      Q.add(p);
    }
    {
      dev::BPassDev p = base(dev::BK_OUTER);
      p.n_tasks = (int)tr0;
      p.oa = x.sa;
      p.ob = x.sb;
      p.dst = psi;
      Q.add(p);
    }
    // a compiled program as SEG passes (transposes are implicit: the other
    // layout's tasks gather columns); dual = the same passes on a second state
    auto add_program = [&](const Compiled& c, const void* src, void* work, void* accum, const void* src2,
                           void* work2) {
      int last_seg = -1;
      for (int k = 0; k < (int)c.launches.size(); ++k)
        if (c.launches[k].kind == Launch::SEG) last_seg = k;
      const void* cur_src = src;
      const void* cur_src2 = src2;
      for (int k = 0; k < (int)c.launches.size(); ++k) {
        const Launch& Lc = c.launches[k];
        if (Lc.kind == Launch::TRANSPOSE) continue;
        if (Lc.kind != Launch::SEG || Lc.cross) throw Error(FFX_EUNSUPPORTED, "batched sector needs a window pass");
        if (Lc.reduce) throw Error(FFX_EUNSUPPORTED, "batched programs do not reduce inside passes");
        dev::BPassDev p = base(dev::BK_SEG);
        p.layout = Lc.layout;
        p.real = Lc.real ? 1 : 0;
        p.n_stages = Lc.n_stages;
        p.stages = Lc.stages;
        const int64_t tasks = Lc.layout == 0 ? tr0 : tr1;
        p.src = cur_src;
        if (k == last_seg && c.final_mode == FINAL_ACCUM) {
          p.mode = dev::SEG_ACCUM;
          p.dst = accum;
        } else if (k == last_seg && c.final_mode == FINAL_NONE) {
          p.mode = dev::SEG_NONE;
        } else {
          p.mode = dev::SEG_STORE;
          p.dst = work;
        }
        p.n_tasks = (int)tasks;
        if (src2) {
          p.src2 = cur_src2;
          p.dst2 = work2;
          p.half = (int)tasks;
          p.n_tasks = (int)(2 * tasks);
        }
        Q.add(p);
        cur_src = work;
        cur_src2 = work2;
      }
    };
    add_program(x.fwd, psi, psi, nullptr, nullptr, nullptr);
    for (int tt = 0; tt <= G.df.L; ++tt) {
      if (tt == 0)
        add_program(x.terms[tt], psi, lam, nullptr, nullptr, nullptr);
      else
        add_program(x.terms[tt], psi, tmp, lam, nullptr, nullptr);
    }
    auto add_sum = [&](double* out, int width, int n_sum) {
      dev::BPassDev p = base(dev::BK_SUM);
      p.n_tasks = 1;
      p.partials = part;
      p.out = out;
      p.width = width;
      p.n_sum = n_sum;
      Q.add(p);
    };
    {
      dev::BPassDev p = base(dev::BK_INNER);
      p.n_tasks = (int)tr0;
      p.src = psi;
      p.src2 = lam;
      p.partials = part;
      p.width = 2;
      Q.add(p);
      add_sum(res, 2, (int)tr0);
    }
    auto add_rdm = [&](double* out) {
      for (int layout = 0; layout < 2; ++layout) {
        dev::BPassDev p = base(dev::BK_RDM);
        p.layout = layout;
        p.n_tasks = (int)(layout == 0 ? td0 : td1);
        p.src = lam;
        p.src2 = psi;
        p.partials = part + (layout == 0 ? 0 : td0 * 2 * NN);
        p.width = 2 * NN;
        Q.add(p);
      }
      add_sum(out, 2 * NN, (int)(td0 + td1));
    };
    for (int k = R - 1; k >= 0; --k) {
      double* Tb = res + 2 + (size_t)k * (4 * NN + 2 * N - 1);
      double* Ta = Tb + 2 * NN;
      double* D = Tb + 4 * NN;
      add_program(x.urot[k], psi, psi, nullptr, lam, lam);
      add_rdm(Tb);
      {
        dev::BPassDev p = base(dev::BK_DGRAD);
        p.n_tasks = (int)tr0;
        p.src = lam;
        p.src2 = psi;
        p.partials = part;
        p.width = 2 * N - 1;
        Q.add(p);
        add_sum(D, 2 * N - 1, (int)tr0);
      }
      add_program(x.udiag[k], psi, psi, nullptr, lam, lam);
      add_rdm(Ta);
    }
  }
  // queue: pass level by pass level; within a level the larger sectors first
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return b.plans[b.inst_type[a]]->elems() > b.plans[b.inst_type[c]]->elems();
  });
  size_t max_levels = 0;
  for (auto& q : ip) max_levels = std::max(max_levels, q.p.size());
  std::vector<dev::BPassDev> all;
  std::vector<int> level_start;  // first pass of each level
  int64_t first = 0;
  for (size_t lv = 0; lv < max_levels; ++lv) {
    level_start.push_back((int)all.size());
    // the passes of a level do not depend on each other: grouped by kind (for
    // the one-launch-per-kind form), instances in size order within a kind
    std::vector<dev::BPassDev> lvl;
    for (int i : order)
      if (lv < ip[i].p.size()) lvl.push_back(ip[i].p[lv]);
    std::stable_sort(lvl.begin(), lvl.end(),
                     [](const dev::BPassDev& a, const dev::BPassDev& c) { return a.kind < c.kind; });
    for (dev::BPassDev p : lvl) {
      p.first = first;
      first += p.n_tasks;
      all.push_back(p);
    }
  }
  level_start.push_back((int)all.size());
  if (queue) {  // the task queue only: nothing is launched
    queue->clear();
    for (size_t lv = 0; lv + 1 < level_start.size(); ++lv)
      for (int pi = level_start[lv]; pi < level_start[lv + 1]; ++pi) {
        const dev::BPassDev& p = all[pi];
        for (int64_t v : {(int64_t)lv, (int64_t)p.inst, (int64_t)p.kind, (int64_t)p.n_tasks, (int64_t)p.need,
                          p.first})
          queue->push_back(v);
      }
    return;
  }
  const dev::BPassDev* d_passes = up.put(all.data(), all.size());
  const int* d_levels = up.put(level_start.data(), level_start.size());
  up.commit();

  // [next, abort, -, -, done per instance..., task counter per level...]
  const size_t n_ctr = (size_t)n + 4 + level_start.size();
  if (b.counters_cap < n_ctr) {
    if (b.counters) (void)hipFree(b.counters);
    b.counters = nullptr;
    b.counters_cap = 0;
    b.counters = (unsigned*)b.dalloc(n_ctr * sizeof(unsigned));
    b.counters_cap = n_ctr;
  }
  HIPCHK(hipMemsetAsync(b.counters, 0, n_ctr * sizeof(unsigned), s));
  dev::BatchDev bd{};
  bd.types = b.d_types;
  bd.passes = d_passes;
  bd.n_passes = (int)all.size();
  bd.n_tasks = first;
  bd.next = b.counters;
  bd.abort = b.counters + 1;
  bd.done = b.counters + 4;
  bd.lds_row_bytes = b.lds_row_bytes;
  bd.max_mt = b.max_mt;
  bd.wq_rows = b.wq_rows;
  if (!b.ev[0]) HIPCHK(hipEventCreate(&b.ev[0]));
  if (!b.ev[1]) HIPCHK(hipEventCreate(&b.ev[1]));
  HIPCHK(hipEventRecord(b.ev[0], s));
  int launches = 0;
  int coop_per_cu = 0, cus = 0;
  if (b.single_launch) {
    coop_per_cu = dev::batch_coop_blocks_per_cu(b.c64, b.lds);
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b.device));
  }
  if (b.single_launch && coop_per_cu >= 1) {  // else (no block fits) one launch per level
    const int per_cu = coop_per_cu;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * cus, first));
    const hipError_t e = dev::batch_launch_coop(b.c64, bd, d_levels, (int)level_start.size() - 1,
                                                b.counters + 4 + n, blocks, b.lds, s);
    if (e != hipSuccess) throw Error(FFX_EDEVICE, std::string("cooperative launch: ") + hipGetErrorString(e));
    check_launch();
    launches = 1;
  } else if (b.persistent) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(b.blocks, first));
    dev::batch_launch(b.c64, bd, blocks, 256, b.lds, s);
    check_launch();
    launches = 1;
  } else {
    for (size_t lv = 0; lv + 1 < level_start.size(); ++lv) {
      for (int p0 = level_start[lv]; p0 < level_start[lv + 1];) {
        int p1 = p0 + 1;
        while (p1 < level_start[lv + 1] && all[p1].kind == all[p0].kind) ++p1;
        const int64_t tasks = (p1 < (int)all.size() ? all[p1].first : first) - all[p0].first;
        if (tasks > 0) {
          dev::batch_launch_kind(b.c64, all[p0].kind, bd, p0, p1, tasks,
                                 dev::batch_lds_for(all[p0].kind, b.lds_row_bytes, b.max_mt, b.wq_rows), s);
          check_launch();
          ++launches;
        }
        p0 = p1;
      }
    }
  }
  HIPCHK(hipEventRecord(b.ev[1], s));
  std::vector<double> hres(res_total);
  unsigned flags[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(hres.data(), results, res_total * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(flags, b.counters, sizeof(flags), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float dms = 0;
  HIPCHK(hipEventElapsedTime(&dms, b.ev[0], b.ev[1]));
  if (kernel_ms) *kernel_ms = dms;
  b.last_device_ms = dms;
  b.last_launches = launches;
  if (flags[1]) throw Error(FFX_EDEVICE, "batched launch stopped: a dependency wait exceeded its bound");
  // ---- host: energies and gradient chain rules --------------------------
  std::vector<size_t> goffs(n + 1, 0);
  for (int i = 0; i < n; ++i) goffs[i + 1] = goffs[i] + (size_t)ffx_lucj_n_params(b.plans[b.inst_type[i]]->norb, ib[i].G->L.R);
  parallel_for(n, [&](int i) {
    const ffx_plan_s& P = *b.plans[b.inst_type[i]];
    const LUCJGrad& G = *ib[i].G;
    const int N = P.norb, NN = N * N, R = G.L.R;
    const double* r = hres.data() + ib[i].res_off;
    energies[i] = r[0];
    std::vector<const double*> Tb(R), Ta(R), D(R);
    for (int k = 0; k < R; ++k) {
      Tb[k] = r + 2 + (size_t)k * (4 * NN + 2 * N - 1);
      Ta[k] = Tb[k] + 2 * NN;
      D[k] = Tb[k] + 4 * NN;
    }
    lucj_grad_assemble(G, N, Tb, Ta, D, grads + goffs[i]);
  });
}

}  // namespace

extern "C" {

int ffx_batch_create(ffx_batch* out, int n_inst, const int* norb, const int* n_alpha, const int* n_beta,
                     ffx_dtype dtype, int device) {
  return guard([&] {
    if (!out || !norb || !n_alpha || !n_beta || n_inst < 1) throw Error(FFX_EINVAL, "bad batch arguments");
    if (dtype != FFX_C128 && dtype != FFX_C64) throw Error(FFX_EINVAL, "unknown dtype");
    *out = nullptr;
    auto b = std::make_unique<ffx_batch_s>();
    b->c64 = dtype == FFX_C64;
    b->device = device;
    b->n_inst = n_inst;
    HIPCHK(hipSetDevice(device));
    std::map<std::tuple<int, int, int>, int> types;
    for (int i = 0; i < n_inst; ++i) {
      auto key = std::make_tuple(norb[i], n_alpha[i], n_beta[i]);
      if (norb[i] < 1 || norb[i] > 16) throw Error(FFX_EUNSUPPORTED, "batched sectors need 1 <= norb <= 16");
      auto it = types.find(key);
      if (it == types.end()) {
        it = types.emplace(key, (int)b->type_key.size()).first;
        b->type_key.push_back(key);
        ffx_plan p = nullptr;
        int rc = ffx_plan_create(&p, norb[i], n_alpha[i], n_beta[i], dtype, device);
        if (rc != FFX_OK) throw Error(rc, last_error());
        b->plans.push_back(p);
        const ffx_plan_s& P = *p;
        for (int cs = 0; cs < 2; ++cs)
          if (P.seg[cs].wt != P.norb || P.seg[cs].Wseg != kernel_window(b->c64))
            throw Error(FFX_EUNSUPPORTED, "batched sector: a row must fit in LDS and norb must be at least the "
                                          "register window (" + std::to_string(kernel_window(b->c64)) + ")");
      }
      b->inst_type.push_back(it->second);
    }
    b->htypes.resize(b->plans.size());
    build_tables(*b);
    *out = b.release();
  });
}

int ffx_batch_destroy(ffx_batch batch) {
  return guard([&] {
    if (!batch) throw Error(FFX_EINVAL, "null batch");
    delete batch;
  });
}

int64_t ffx_batch_workspace_bytes(ffx_batch batch) {
  if (!batch) return -1;
  int64_t s = 0;
  for (int i = 0; i < batch->n_inst; ++i) s += 3 * (int64_t)state_bytes(*batch, i);
  return s;
}

int ffx_batch_lucj_energy_grad(ffx_batch batch, const ffx_lucj* ops, const ffx_df_ham* hams, double* energies,
                               double* grads, void* workspace, void* stream) {
  return guard([&] {
    if (!batch || !ops || !hams || !energies || !grads || !workspace) throw Error(FFX_EINVAL, "null pointer");
    HIPCHK(hipSetDevice(batch->device));
    const auto t0 = std::chrono::steady_clock::now();
    run_batch(*batch, ops, hams, energies, grads, workspace, (hipStream_t)stream, nullptr);
    batch->last_call_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
}

int ffx_batch_tune(ffx_batch batch, const ffx_lucj* ops, const ffx_df_ham* hams, void* workspace, void* stream,
                   int* target_elems, int* stage_rots) {
  return guard([&] {
    if (!batch || !ops || !hams || !workspace) throw Error(FFX_EINVAL, "null pointer");
    ffx_batch_s& b = *batch;
    HIPCHK(hipSetDevice(b.device));
    std::vector<double> e(b.n_inst);
    size_t ng = 0;
    for (int i = 0; i < b.n_inst; ++i) ng += (size_t)ffx_lucj_n_params(ops[i].norb, ops[i].n_reps);
    std::vector<double> g(ng);
    int best_t = b.target_elems, best_r = b.stage_rots;
    float best = 1e30f;
    for (int tgt : {1024, 2048, 3072, 4096, 6144, 8192, 16384}) {
      b.target_elems = tgt;
      try {
        build_tables(b);
      } catch (const Error&) {
        continue;  // does not fit in LDS
      }
      for (int rots : {16, 64}) {
        b.stage_rots = rots;
        float ms = 0, m2 = 0;
        run_batch(b, ops, hams, e.data(), g.data(), workspace, (hipStream_t)stream, &ms);  // warm
        run_batch(b, ops, hams, e.data(), g.data(), workspace, (hipStream_t)stream, &m2);
        if (m2 < best) {
          best = m2;
          best_t = tgt;
          best_r = rots;
        }
      }
    }
    b.target_elems = best_t;
    b.stage_rots = best_r;
    build_tables(b);
    if (target_elems) *target_elems = best_t;
    if (stage_rots) *stage_rots = best_r;
  });
}

int ffx_batch_timing(ffx_batch batch, double* device_ms, double* call_ms, int* launches) {
  return guard([&] {
    if (!batch) throw Error(FFX_EINVAL, "null batch");
    if (device_ms) *device_ms = batch->last_device_ms;
    if (call_ms) *call_ms = batch->last_call_ms;
    if (launches) *launches = batch->last_launches;
  });
}

int ffx_batch_single_launch(ffx_batch batch, int enable) {
  return guard([&] {
    if (!batch) throw Error(FFX_EINVAL, "null batch");
    batch->single_launch = enable != 0;
  });
}

int ffx_batch_queue(ffx_batch batch, const ffx_lucj* ops, const ffx_df_ham* hams, void* workspace, void* stream,
                    int64_t* table, int64_t cap, int64_t* n_passes) {
  return guard([&] {
    if (!batch || !ops || !hams || !workspace || !n_passes) throw Error(FFX_EINVAL, "null pointer");
    HIPCHK(hipSetDevice(batch->device));
    std::vector<int64_t> q;
    std::vector<double> e(batch->n_inst);
    size_t ng = 0;
    for (int i = 0; i < batch->n_inst; ++i) ng += (size_t)ffx_lucj_n_params(ops[i].norb, ops[i].n_reps);
    std::vector<double> g(ng);
    run_batch(*batch, ops, hams, e.data(), g.data(), workspace, (hipStream_t)stream, nullptr, &q);
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    *n_passes = (int64_t)(q.size() / 6);
    if (table) {
      if (cap < *n_passes) throw Error(FFX_EINVAL, "queue table too small");
      std::copy(q.begin(), q.end(), table);
    }
  });
}

int ffx_batch_persistent(ffx_batch batch, int enable) {
  return guard([&] {
    if (!batch) throw Error(FFX_EINVAL, "null batch");
    if (enable) throw Error(FFX_EUNSUPPORTED, "the task-queue persistent launch is switched off");
    batch->persistent = false;
  });
}

int ffx_batch_info(ffx_batch batch, int* target_elems, int* stage_rots, int* blocks, int64_t* lds_bytes) {
  return guard([&] {
    if (!batch) throw Error(FFX_EINVAL, "null batch");
    if (target_elems) *target_elems = batch->target_elems;
    if (stage_rots) *stage_rots = batch->stage_rots;
    if (blocks) *blocks = batch->blocks;
    if (lds_bytes) *lds_bytes = (int64_t)batch->lds;
  });
}

}  // extern "C"
