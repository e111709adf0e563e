// Gate-program compiler and executor.
//
// A program is a sequence of orbital rotations (each split into its alpha and
// beta Givens decompositions) and diagonal operations.  It is executed as
// alternating "visits" to the two spins: the state is read row-wise, so the
// rotations of the column spin of the current layout run inside segment
// passes; when a diagonal operation needs the other spin's pending rotations,
// the state is transposed and the roles swap.  Within a visit, Givens
// rotations that stay inside the segment window become register-window stages
// of a segment pass; rotations that cross segments run as whole-spin window
// passes between segment passes.  The phase layer that ends each Givens
// decomposition is diagonal, so it is deferred into the next diagonal phase
// stage (or a final phase stage) instead of costing a pass of its own.
#include <cmath>
#include <cstdlib>
#include <deque>
#include <map>
#include <mutex>

#include "plan.h"

namespace ffx {

namespace {

struct Pending {
  bool has = false;
  bool sign_only = true;
  uint32_t sign = 0;
  std::vector<double> delta;
};

struct Item {
  int kind = 0;  // 0: Givens part, 1: diagonal stage
  const Decomposition* d = nullptr;
  dev::StageDev st{};
};

std::vector<std::vector<int>> rotation_deps(const std::vector<Givens>& rots, int norb) {
  std::vector<std::vector<int>> deps(rots.size());
  std::vector<int> last(norb, -1);
  for (size_t i = 0; i < rots.size(); ++i) {
    int p = rots[i].p;
    for (int q : {p, p + 1})
      if (last[q] >= 0) deps[i].push_back(last[q]);
    last[p] = last[p + 1] = (int)i;
  }
  return deps;
}

// rotations inside [a, a + w) whose predecessors are all done or taken, in order
std::vector<int> take_window(const std::vector<Givens>& rots, const std::vector<std::vector<int>>& deps,
                             const std::vector<char>& done, int a, int w) {
  std::vector<char> taken(rots.size(), 0);
  std::vector<int> out;
  for (size_t i = 0; i < rots.size(); ++i) {
    if (done[i]) continue;
    int p = rots[i].p;
    if (p < a || p + 1 >= a + w) continue;
    bool ok = true;
    for (int d : deps[i])
      if (!done[d] && !taken[d]) {
        ok = false;
        break;
      }
    if (ok) {
      taken[i] = 1;
      out.push_back((int)i);
    }
  }
  return out;
}

// The order in which a decomposition's rotations are applied: register-window
// stages inside the segment window, a rotation on the pair straddling the
// segment window (applied as the next segment pass loads), or a whole-spin
// window pass.  It depends only on the positions of the rotations and the
// window parameters, so it is computed once per structure and reused (every
// decomposition of an N-orbital rotation has the same positions).
constexpr int kScheduleBeam = 300;  // partial schedules kept by the stage search

struct SchedStep {
  int kind;  // 0: segment-pass stage at window a; 1: crossing rotation idx[0]; 2: whole-spin window pass at a
  int a;
  std::vector<int> idx;
};

const std::vector<SchedStep>& rotation_schedule(const std::vector<Givens>& rots, int N, int wseg, int wt, int W,
                                                int cap, bool cross) {
  static std::mutex mu;
  static std::map<std::vector<int>, std::vector<SchedStep>> cache;
  std::vector<int> key{N, wseg, wt, W, cap, cross ? 1 : 0};
  for (const Givens& g : rots) key.push_back(g.p);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  std::vector<SchedStep> out;
  // no rotation crosses the segment window: the searched schedule (fewer
  // stages than the greedy one for some sizes, e.g. 12 instead of 13 at 16
  // orbitals)
  int max_p = -1;
  for (const Givens& g : rots) max_p = std::max(max_p, g.p);
  if (wseg >= 2 && max_p + 2 <= wt) {
    bool fits = true;
    for (const Pass& ps : schedule_windows_beam(rots, wt, wseg, kScheduleBeam)) {
      if ((int)ps.idx.size() > cap) fits = false;
      out.push_back(SchedStep{0, ps.a, ps.idx});
    }
    if (fits) return cache.emplace(std::move(key), std::move(out)).first->second;
    out.clear();
  }
  // rotations cross the segment window and none is applied at load: stages
  // and whole-spin window passes from the cost search (a window pass counted
  // as three stages, about its time against a stage's at 18 orbitals).  At 18
  // orbitals with plane segments it needs 14 stages per decomposition where
  // the greedy order below needs 16; at 32 orbitals with ten above the
  // segment window, 46 stages and 8 window passes where the greedy order
  // needs 55 and 8.  Its host time grows quickly with the rotation count
  // (once per rotation structure): the full beam up to 20 orbitals (0.1 s at
  // 18), a narrower one up to 32 (0.4 s).
  // a stage with straight-line code (one of the stage shapes) counts 1, any other 2
  const std::function<bool(const std::vector<int>&)> shaped = [](const std::vector<int>& pos) {
    for (int k = 0; k < dev::kNumShapes; ++k) {
      if ((int)pos.size() != dev::kShapeLen[k]) continue;
      bool same = true;
      for (size_t i = 0; i < pos.size() && same; ++i) same = pos[i] == dev::kShapeP[k][i];
      if (same) return true;
    }
    return false;
  };
  const auto* shaped_p = wseg == dev::kShapeW ? &shaped : nullptr;
  const int beam = N <= 20 ? kScheduleBeam : 60;
  if (wseg >= 2 && !cross && N <= 32) {
    const std::vector<SchedPass> sp = schedule_windows_cross(rots, N, wt, wseg, W, beam, 3, shaped_p);
    bool ok = !sp.empty();
    for (const SchedPass& p : sp) ok = ok && (int)p.idx.size() <= cap;
    if (ok) {
      for (const SchedPass& p : sp) out.push_back(SchedStep{p.win ? 2 : 0, p.a, p.idx});
      return cache.emplace(std::move(key), std::move(out)).first->second;
    }
  }
  // the rotation on the pair straddling the segment window applied at load:
  // the same search with that pair as the only "window pass" (a two-orbital
  // window at wt - 1, which holds one ready rotation at a time); at 16
  // orbitals with half rows, 12 stages per decomposition, all with
  // straight-line code, where the greedy order below needs 13.  (Rotations
  // above the pair, which need window passes, leave the search without a
  // schedule.)
  if (wseg >= 2 && cross && N <= 32) {
    const std::vector<SchedPass> sp = schedule_windows_cross(rots, N, wt, wseg, 2, beam, 3, shaped_p);
    bool ok = !sp.empty();
    for (const SchedPass& p : sp)
      ok = ok && (int)p.idx.size() <= cap && (!p.win || (p.idx.size() == 1 && rots[p.idx[0]].p == wt - 1));
    if (ok) {
      for (const SchedPass& p : sp) out.push_back(p.win ? SchedStep{1, 0, p.idx} : SchedStep{0, p.a, p.idx});
      return cache.emplace(std::move(key), std::move(out)).first->second;
    }
  }
  const auto deps = rotation_deps(rots, N);
  std::vector<char> done(rots.size(), 0);
  size_t n_done = 0;
  while (n_done < rots.size()) {
    while (wseg >= 2) {
      int best_a = -1;
      std::vector<int> best;
      for (int a = 0; a + wseg <= wt; ++a) {
        auto t = take_window(rots, deps, done, a, wseg);
        if (t.size() > best.size()) {
          best = t;
          best_a = a;
        }
      }
      if (best.empty()) break;
      // a stage's rotations are spread over the 64 lanes of a wave; the taken
      // list is in dependency order, so any prefix is a valid stage
      if (best.size() > (size_t)cap) best.resize(cap);
      for (int i : best) done[i] = 1;
      n_done += best.size();
      out.push_back(SchedStep{0, best_a, best});
    }
    if (n_done == rots.size()) break;
    if (cross) {
      int xi = -1;
      for (size_t i = 0; i < rots.size() && xi < 0; ++i) {
        if (done[i] || rots[i].p != wt - 1) continue;
        bool ready = true;
        for (int dp : deps[i]) ready = ready && done[dp];
        if (ready) xi = (int)i;
      }
      if (xi >= 0) {
        done[xi] = 1;
        ++n_done;
        out.push_back(SchedStep{1, 0, {xi}});
        continue;
      }
    }
    int best_a = -1;
    std::vector<int> best;
    for (int a = 0; a + W <= N; ++a) {
      auto t = take_window(rots, deps, done, a, W);
      if (t.size() > best.size()) {
        best = t;
        best_a = a;
      }
    }
    if (best.empty()) throw Error(FFX_EDEVICE, "rotation schedule made no progress");
    for (int i : best) done[i] = 1;
    n_done += best.size();
    out.push_back(SchedStep{2, best_a, best});
  }
  return cache.emplace(std::move(key), std::move(out)).first->second;
}

// index of the stage shape whose position list equals the stage's, or -1
int stage_shape(const std::vector<dev::RotDev>& rots, int w) {
  if (w != dev::kShapeW) return -1;
  for (int k = 0; k < dev::kNumShapes; ++k) {
    if ((int)rots.size() != dev::kShapeLen[k]) continue;
    bool same = true;
    for (size_t i = 0; i < rots.size() && same; ++i) same = rots[i].p == dev::kShapeP[k][i];
    if (same) return k;
  }
  return -1;
}

}  // namespace

Compiled compile_program(ffx_plan_s& P, Upload& up, const Program& prog, int final_mode, hipStream_t s) {
  Compiled c;
  c.final_mode = final_mode;
  const int N = P.norb;
  const int64_t da = P.dim[0], db = P.dim[1];

  // arena: per diagonal function the tables A (alpha strings) and B (beta
  // strings), then one complex column-factor table per phase stage
  size_t n_phase = 2;
  for (const ProgOp& op : prog.ops) n_phase += (op.kind == ProgOp::PHASE || op.kind == ProgOp::ROT) ? 1 : 0;
  const size_t dmax = (size_t)std::max(da, db);
  const size_t arena_need = prog.diags.size() * (size_t)(da + db) + n_phase * 2 * dmax;
  double* arena = P.arena_hook ? P.arena_hook(P.arena_ctx, arena_need) : P.arena_for(arena_need, s);
  size_t arena_off = prog.diags.size() * (size_t)(da + db);
  std::vector<const double*> Cd(prog.diags.size(), nullptr), CTd(prog.diags.size(), nullptr);
  for (size_t i = 0; i < prog.diags.size(); ++i) {
    const DiagSpec& d = prog.diags[i];
    TableBuild tb{};
    if (d.lin_a) tb.spec.lin_a = up.put(d.lin_a, N);
    if (d.lin_b) tb.spec.lin_b = up.put(d.lin_b, N);
    if (d.Qa) tb.spec.Qa = up.put(d.Qa, (size_t)N * N);
    if (d.Qb) tb.spec.Qb = up.put(d.Qb, (size_t)N * N);
    tb.A = arena + i * (size_t)(da + db);
    tb.B = tb.A + da;
    c.tables.push_back(tb);
    if (d.C) {
      std::vector<double> CT((size_t)N * N);
      for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q) CT[q * N + p] = d.C[p * N + q];
      Cd[i] = up.put(d.C, (size_t)N * N);
      CTd[i] = up.put(CT.data(), CT.size());
    }
  }

  int layout = 0;
  std::vector<const Decomposition*> pending_other;
  Pending pend[2];
  std::vector<Item> visit;
  auto colspin = [&]() { return layout == 0 ? 1 : 0; };
  auto rowspin = [&]() { return layout == 0 ? 0 : 1; };

  // A phase stage: the column-only factor goes into a per-stage table built on
  // the device; deferred orbital phase layers of the row spin go into drow /
  // sign_row and those of the column spin into the column table.
  auto phase_stage = [&](int diag, double scale) {
    dev::StageDev st{};
    st.type = dev::ST_PHASE;
    st.scale = scale;
    const int cs = colspin();
    ColfBuild cb{};
    cb.spin = cs;
    cb.scale = scale;
    if (diag >= 0) {
      const TableBuild& tb = c.tables[diag];
      st.A = layout == 0 ? tb.A : tb.B;
      st.C = layout == 0 ? Cd[diag] : CTd[diag];
      cb.B = layout == 0 ? tb.B : tb.A;
    }
    for (int role = 0; role < 2; ++role) {
      const int sp = role == 0 ? rowspin() : cs;
      Pending& pd = pend[sp];
      if (!pd.has) continue;
      if (role == 0) {
        if (pd.sign_only)
          st.sign_row ^= pd.sign;
        else
          st.drow = up.put(pd.delta.data(), pd.delta.size());
      } else {
        if (pd.sign_only)
          cb.sign ^= pd.sign;
        else
          cb.delta = up.put(pd.delta.data(), pd.delta.size());
      }
      pd = Pending{};
    }
    if (!cb.B && !cb.delta && cb.sign) {
      st.sign_col = cb.sign;  // signs alone: taken from each column's mask
    } else if (cb.B || cb.delta || cb.sign) {
      const size_t n = (size_t)P.dim[cs];
      if (arena_off + 2 * n > arena_need) throw Error(FFX_EUNSUPPORTED, "diagonal table arena exhausted");
      cb.out = arena + arena_off;
      arena_off += 2 * n;
      c.colfs.push_back(cb);
      st.colf = cb.out;
    }
    return st;
  };
  auto diag_stage = [&](int type, int diag) {
    dev::StageDev st{};
    st.type = type;
    if (diag >= 0) {
      const TableBuild& tb = c.tables[diag];
      st.A = layout == 0 ? tb.A : tb.B;
      st.B = layout == 0 ? tb.B : tb.A;
      st.C = layout == 0 ? Cd[diag] : CTd[diag];
    }
    return st;
  };
  auto add_givens = [&](const Decomposition* d) {
    const int sp = colspin();
    if (pend[sp].has) {  // an earlier phase layer of this spin must land first
      Item it;
      it.kind = 1;
      it.st = phase_stage(-1, 0.0);
      visit.push_back(it);
    }
    Item it;
    it.kind = 0;
    it.d = d;
    if (!d->rots.empty()) visit.push_back(it);
    Pending& pd = pend[sp];
    for (double x : d->phase)
      if (x != 0.0) pd.has = true;
    if (pd.has) {
      pd.sign_only = d->real;
      if (d->real) {
        pd.sign = 0;
        for (int p = 0; p < N; ++p)
          if (d->phase[p] != 0.0) pd.sign |= 1u << p;
      } else {
        pd.delta = d->phase;
      }
    }
  };

  auto close_visit = [&](bool force_seg) {
    // a visit whose Givens rotations are all real holds each row as two planes
    // where the plan has them (whole rows: no crossing rotation, one pass)
    bool planes = P.plane[colspin()].n_seg > 0;
    {
      bool any_rot = false;
      for (const Item& it : visit)
        if (it.kind == 0) {
          any_rot = true;
          if (!it.d->real) planes = false;
        }
      planes = planes && any_rot;
    }
    const auto& ss = planes ? P.plane[colspin()] : P.seg[colspin()];
    const int64_t n_rows = layout == 0 ? da : db;
    const int ncol = P.n[colspin()];
    const double pairs_per_row = (double)binom(N - 2, ncol - 1);
    std::vector<dev::StageDev> stages;
    Launch cur{};
    cur.kind = Launch::SEG;
    cur.layout = layout;
    cur.planes = planes;
    bool any = false;
    auto flush_seg = [&](bool force) {
      if (stages.empty() && !force && !cur.cross) return;
      cur.stages = stages.empty() ? nullptr : up.put(stages.data(), stages.size());
      cur.n_stages = (int)stages.size();
      c.launches.push_back(cur);
      stages.clear();
      cur = Launch{};
      cur.kind = Launch::SEG;
      cur.layout = layout;
      cur.planes = planes;
    };
    for (const Item& it : visit) {
      if (it.kind == 1) {
        stages.push_back(it.st);
        if (it.st.type == dev::ST_REDUCE) cur.reduce = true;
        any = true;
        continue;
      }
      const Decomposition& d = *it.d;
      const double K = 0.5 * N * (N - 1);
      const int cap = std::max(1, std::min(P.max_stage_rots, dev::kMaxStageRots));
      for (const SchedStep& step : rotation_schedule(d.rots, N, ss.Wseg, ss.wt, P.W, cap, ss.cross)) {
        const double slots = (double)step.idx.size() * pairs_per_row * (double)n_rows * (d.real ? 8.0 : 12.0);
        if (step.kind == 1) {
          // starts the next segment pass: applied as the segments are loaded
          flush_seg(false);
          const Givens& g = d.rots[step.idx[0]];
          if (!(g.c >= 0.0)) throw Error(FFX_EDEVICE, "Givens rotation with a negative cosine");
          cur.cross = true;
          cur.cross_rot = dev::make_rot(0, g.c, g.s.real(), g.s.imag());
          cur.valu_slots += slots;
          cur.rot_sides += 1.0 / K;
          continue;
        }
        std::vector<dev::RotDev> buf;
        for (int i : step.idx) {
          const Givens& g = d.rots[i];
          // the shear form of a real rotation needs c >= 0, which every
          // decomposition's rotation has (c = |b| / r)
          if (!(g.c >= 0.0)) throw Error(FFX_EDEVICE, "Givens rotation with a negative cosine");
          buf.push_back(dev::make_rot(g.p - step.a, g.c, g.s.real(), g.s.imag()));
        }
        if (step.kind == 0) {
          dev::StageDev st{};
          st.type = dev::ST_GIVENS;
          st.a = step.a;
          st.nrot = (int)buf.size();
          st.shape = stage_shape(buf, ss.Wseg);
          st.rots = up.put(buf.data(), buf.size());
          stages.push_back(st);
          cur.real = cur.real && d.real;
          cur.valu_slots += slots;
          cur.rot_sides += step.idx.size() / K;
          any = true;
        } else {
          // other rotations crossing segments: one whole-spin window pass
          flush_seg(false);
          Launch w{};
          w.kind = Launch::WIN;
          w.layout = layout;
          w.real = d.real;
          w.a = step.a;
          w.nrot = (int)buf.size();
          w.rots = up.put(buf.data(), buf.size());
          w.valu_slots = slots;
          w.rot_sides = step.idx.size() / K;
          c.launches.push_back(w);
        }
      }
    }
    flush_seg(force_seg && !any);
    if (!stages.empty()) flush_seg(false);
    visit.clear();
  };
  auto transpose = [&]() {
    Launch t{};
    t.kind = Launch::TRANSPOSE;
    t.layout = layout;
    c.launches.push_back(t);
    layout ^= 1;
  };
  auto switch_layout = [&]() {
    close_visit(false);
    transpose();
    for (const Decomposition* d : pending_other) add_givens(d);
    pending_other.clear();
  };

  // Rotations with c = 1 and s = 0 are exact identities and leave the
  // program; so does an orbital rotation with no rotation and no phase left
  // (for example the identity basis change of a diagonal-only term).
  std::deque<Decomposition> pruned;
  auto prune = [&](const Decomposition* d) -> const Decomposition* {
    bool ident = false, phase = false;
    for (const Givens& g : d->rots)
      if (g.c == 1.0 && g.s == cd(0.0, 0.0)) ident = true;
    for (double x : d->phase)
      if (x != 0.0) phase = true;
    if (!ident) return d;
    Decomposition q;
    q.real = d->real;
    q.phase = d->phase;
    for (const Givens& g : d->rots)
      if (!(g.c == 1.0 && g.s == cd(0.0, 0.0))) q.rots.push_back(g);
    if (q.rots.empty() && !phase) return nullptr;
    pruned.push_back(std::move(q));
    return &pruned.back();
  };
  for (const ProgOp& op : prog.ops) {
    if (op.kind == ProgOp::ROT) {
      const Decomposition* dc = prune(op.part[colspin()]);
      const Decomposition* dr = prune(op.part[rowspin()]);
      if (dc) add_givens(dc);
      if (dr) pending_other.push_back(dr);
      continue;
    }
    if (!pending_other.empty()) switch_layout();
    Item it;
    it.kind = 1;
    if (op.kind == ProgOp::PHASE) {
      it.st = phase_stage(op.diag, op.scale);
    } else if (op.kind == ProgOp::SCALE) {
      it.st = diag_stage(dev::ST_SCALE, op.diag);
    } else {
      it.st = diag_stage(dev::ST_REDUCE, op.diag);
    }
    visit.push_back(it);
    if (op.kind == ProgOp::REDUCE) {
      // close now, so that the reduction's partial sums belong to one launch
      close_visit(false);
      c.launches.back().reduce_out = op.out;
    }
  }
  if (!pending_other.empty()) switch_layout();
  if (final_mode != FINAL_NONE && (pend[0].has || pend[1].has)) {
    Item it;
    it.kind = 1;
    it.st = phase_stage(-1, 0.0);
    visit.push_back(it);
  }
  close_visit(false);
  if (final_mode != FINAL_NONE && layout == 1) transpose();
  if (final_mode == FINAL_ACCUM &&
      (c.launches.empty() || c.launches.back().kind != Launch::SEG || c.launches.back().layout != 0))
    close_visit(true);  // a stage-free segment pass that adds the result into the target
  // A transpose after a segment pass that stores the state: the pass stores
  // its rows as columns of the new layout instead (scatter); otherwise, a
  // transpose followed by a segment pass of the new layout: the pass gathers
  // its rows from the old layout (gather).  Either saves one state round trip.
  // Measured on the DF step at 16 orbitals, complex128: gathering 2 % faster
  // than the transposes (eight amplitudes of a cache line serve eight blocks
  // of one XCD), scattering 2 % faster than gathering; complex64: gathering
  // 1.5 % slower than the transposes (sixteen blocks per line), scattering
  // 0.5 % slower, so complex64 keeps the transposes.
  // FFX_SCATTER=0/1 and FFX_GATHER=0/1 override the choices (measurements).
  bool scatter = !P.c64;
  if (const char* e = std::getenv("FFX_SCATTER")) scatter = std::atoi(e) != 0;
  bool gather = !P.c64;
  if (const char* e = std::getenv("FFX_GATHER")) gather = std::atoi(e) != 0;
  int last_seg = -1;
  for (int i = 0; i < (int)c.launches.size(); ++i)
    if (c.launches[i].kind == Launch::SEG) last_seg = i;
  std::vector<Launch> fused;
  for (size_t i = 0; i < c.launches.size(); ++i) {
    const Launch& L = c.launches[i];
    // (the last segment pass of a program without a final state stores nothing)
    if (scatter && L.kind == Launch::TRANSPOSE && !fused.empty() && fused.back().kind == Launch::SEG &&
        !fused.back().scatter && !((int)i - 1 == last_seg && final_mode == FINAL_NONE)) {
      fused.back().scatter = true;
      continue;
    }
    if (gather && L.kind == Launch::TRANSPOSE && i + 1 < c.launches.size() &&
        c.launches[i + 1].kind == Launch::SEG) {
      Launch nx = c.launches[i + 1];
      nx.gather = true;
      fused.push_back(nx);
      ++i;
      continue;
    }
    fused.push_back(L);
  }
  c.launches = std::move(fused);
  return c;
}

void execute_program(ffx_plan_s& P, const Compiled& c, const void* src, void* work, void* accum,
                     hipStream_t s) {
  const int64_t da = P.dim[0], db = P.dim[1];
  const int N = P.norb;
  for (const TableBuild& tb : c.tables) {
    dev::diag_tables(P.d_masks[0], da, P.d_masks[1], db, N, tb.spec, tb.A, tb.B, nullptr, s);
    check_launch();
  }
  for (const ColfBuild& cb : c.colfs) {
    dev::column_factors(P.d_masks[cb.spin], P.dim[cb.spin], cb.B, cb.scale, cb.delta, cb.sign, cb.out, s);
    check_launch();
  }
  int last_seg = -1;
  for (int i = 0; i < (int)c.launches.size(); ++i)
    if (c.launches[i].kind == Launch::SEG) last_seg = i;
  const void* cur_src = src;
  void* cur = work;
  if (src != work && (c.launches.empty() || c.launches[0].kind != Launch::SEG)) {
    HIPCHK(hipMemcpyAsync(work, src, P.state_bytes(), hipMemcpyDeviceToDevice, s));
    cur_src = work;
  }
  const bool square = da == db;
  // Buffers: a segment pass with a crossing rotation must not write the
  // buffer it reads, so it moves the state to the other of (work, tmp); a
  // non-square transpose does as well.  When the state would end in tmp, one
  // in-place segment pass moves it too, so that it ends in work.
  const int nl = (int)c.launches.size();
  std::vector<char> move(nl, 0);
  auto simulate = [&]() {
    bool at_src = src != work && nl > 0 && c.launches[0].kind == Launch::SEG;
    bool in_work = true;  // where cur points
    int last_plain = -1;
    for (int i = 0; i < nl; ++i) {
      const Launch& L = c.launches[i];
      const bool store = L.kind == Launch::SEG && !(i == last_seg && c.final_mode != FINAL_STORE);
      if (L.kind == Launch::SEG) {
        if (store && !at_src && (L.cross || L.gather || L.scatter || move[i])) in_work = !in_work;
        if (store && !at_src && !L.cross && !L.gather && !L.scatter) last_plain = i;
        at_src = false;
      } else if (L.kind == Launch::TRANSPOSE && !square) {
        in_work = !in_work;
      }
    }
    return std::make_pair(in_work, last_plain);
  };
  if (c.final_mode == FINAL_STORE) {
    auto r = simulate();
    if (!r.first && r.second >= 0) move[r.second] = 1;
  }
  for (int i = 0; i < (int)c.launches.size(); ++i) {
    const Launch& L = c.launches[i];
    const int64_t rows = L.layout == 0 ? da : db;
    const int64_t cols = L.layout == 0 ? db : da;
    const int cs = L.layout == 0 ? 1 : 0;
    ffx_plan_s::Timed tm{};
    const bool timed = P.timing && (L.kind == Launch::SEG || L.kind == Launch::WIN);
    if (timed) {
      tm.a = P.take_event();
      tm.b = P.take_event();
      tm.kind = L.kind == Launch::SEG ? (L.planes ? 2 : 1) : 0;
      tm.spin = cs;
      tm.valu_slots = L.valu_slots;
      tm.alg_bytes = L.rot_sides * 2.0 * (double)P.state_bytes();
      HIPCHK(hipEventRecord(tm.a, s));
    }
    if (L.kind == Launch::SEG) {
      const auto& ss = L.planes ? P.plane[cs] : P.seg[cs];
      dev::SegPassDev p{};
      p.src = cur_src;
      p.norb = N;
      p.n_rows = rows;
      p.row_len = cols;
      p.row_masks = P.d_masks[L.layout == 0 ? 0 : 1];
      p.col_masks = P.d_masks[cs];
      p.n_seg = ss.n_seg;
      p.segs = ss.d_segs;
      p.n_stages = L.n_stages;
      p.stages = L.stages;
      p.partials = L.reduce ? P.partials : nullptr;
      p.lds_row_bytes = (int)(((size_t)ss.max_len * (L.planes ? 8 : P.elem()) + 15) & ~(size_t)15);
      p.max_mt = ss.max_mt;
      if (L.cross) {
        p.cross = 1;
        p.cross_c = L.cross_rot.c;
        p.cross_sr = L.cross_rot.sr;
        p.cross_si = L.cross_rot.si;
      }
      if (L.gather) p.gather = 1;
      if (L.scatter) p.scatter = 1;
      if (L.gather || L.scatter || L.cross) p.xcd_rows = (rows + 7) / 8;
      if (i == last_seg && c.final_mode == FINAL_ACCUM) {
        p.mode = dev::SEG_ACCUM;
        p.dst = accum;
      } else if (i == last_seg && c.final_mode == FINAL_NONE) {
        p.mode = dev::SEG_NONE;
        p.dst = nullptr;
      } else {
        p.mode = dev::SEG_STORE;
        if (cur_src == cur && (L.cross || L.gather || L.scatter || move[i]))
          cur = (cur == work) ? P.tmp_state() : work;
        p.dst = cur;
      }
      if ((L.cross || L.gather || L.scatter) && p.dst == p.src)
        throw Error(FFX_EDEVICE, "crossing rotation, gathering or scattering pass needs an out-of-place pass");
      if (L.planes)
        dev::seg_pass_planes(ss.Wseg, ss.threads, p, ss.lds, s);
      else
        dev::seg_pass(P.c64, L.real, ss.Wseg, p, ss.threads, ss.lds, s);
      check_launch();
      if (L.reduce) {
        dev::sum_partials(P.partials, (int)(rows * ss.n_seg), L.reduce_out, s);
        check_launch();
      }
      cur_src = cur;
    } else if (L.kind == Launch::WIN) {
      dev::win_pass(P.c64, L.real, 1, cur, rows, cols, P.win[cs][L.a], L.rots, L.nrot, nullptr, s);
      check_launch();
      cur_src = cur;
    } else if (L.kind == Launch::TRANSPOSE) {
      if (square) {
        dev::transpose_square(P.c64, cur, rows, s);
      } else {
        void* other = (cur == work) ? P.tmp_state() : work;
        dev::transpose(P.c64, cur, other, rows, cols, s);
        cur = other;
      }
      check_launch();
      cur_src = cur;
    }
    if (timed) {
      HIPCHK(hipEventRecord(tm.b, s));
      P.timed.push_back(tm);
    }
  }
  if (c.final_mode == FINAL_STORE && cur != work)
    HIPCHK(hipMemcpyAsync(work, cur, P.state_bytes(), hipMemcpyDeviceToDevice, s));
}

}  // namespace ffx
