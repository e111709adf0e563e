// C ABI of libffx (include/ffx.h): plans, parameter upload, gate programs and
// the DF-Trotter / LUCJ / energy / adjoint-gradient drivers.  Every step on
// the state runs in the HIP kernels of kernels.hip; this file only prepares
// small FP64 host data (Givens decompositions, eigendecompositions, Slater
// column minors, gradient chain rules) and enqueues launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "device.h"
#include "ffx.h"
#include "host.h"
#include "plan.h"
#include "drivers.h"

using namespace ffx;

namespace ffx {
void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(FFX_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}
}  // namespace ffx

namespace {

void validate_plan(ffx_plan plan) {
  if (!plan) throw Error(FFX_EINVAL, "null plan");
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// Transition one-body matrix of lam and psi, both spins:
//   Tout[0 .. 2N^2) alpha part, Tout[2N^2 .. 4N^2) beta part (interleaved complex)
// For norb <= 16 the excitations are taken inside rows on the matrix cores
// (beta on the alpha-major states, alpha on their transposes); otherwise
// between row pairs.

static_assert(kCodeMoffBits == dev::kCodeMoffBitsDev, "class code fields differ between host and device");

void ensure_rank_tables(ffx_plan_s& P) {
  if (P.rank_lo) return;
  std::vector<int> lo(256, 0), hi(256 * 17, 0);
  for (int v = 0; v < 256; ++v) {
    int t = 0;
    for (int j = 0; j < 8; ++j)
      if ((v >> j) & 1) lo[v] += (int)binom(j, ++t);
    for (int c = 0; c <= 16; ++c) {
      int u = c, acc = 0;
      for (int j = 0; j < 8; ++j)
        if ((v >> j) & 1) acc += (int)binom(8 + j, ++u);
      hi[v * 17 + c] = acc;
    }
  }
  // published only once both tables are on the device (a failure in between
  // leaves the plan without them, to be built by the next call)
  int* dlo = (int*)P.dalloc(lo.size() * 4);
  int* dhi = (int*)P.dalloc(hi.size() * 4);
  HIPCHK(hipMemcpy(dlo, lo.data(), lo.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dhi, hi.data(), hi.size() * 4, hipMemcpyHostToDevice));
  P.rank_lo = dlo;
  P.rank_hi = dhi;
}

// The (n-1)-electron strings K of column spin cs for the matrix-core kernel,
// grouped by their occupation of the top norb - nlow orbitals, with nlow the
// largest value whose home column ranges (strings with the group's top
// occupation) of two states and the group's K list fit the LDS budget.
void ensure_rdm_strings(ffx_plan_s& P, int cs) {
  auto& R = P.rdm_k[cs];
  if (R.ready) return;
  const int N = P.norb, n = P.n[cs];
  const auto& str = P.str[cs];
  std::vector<uint32_t> K;
  if (n >= 1)
    for (uint32_t m = 0; m < (1u << N); ++m)
      if (__builtin_popcount(m) == n - 1) K.push_back(m);
  const size_t budget = 140 * 1024;
  for (int h = 0; h <= N; ++h) {
    const int nlow = N - h;
    std::vector<int> group;
    std::vector<uint32_t> sorted;
    int max_home = 0, max_inter = 0;
    for (uint32_t H = 0; H < (1u << h); ++H) {
      std::vector<uint32_t> ks;
      for (uint32_t k : K)
        if ((k >> nlow) == H) ks.push_back(k);
      if (ks.empty()) continue;
      int first = -1, cnt = 0;
      for (size_t i = 0; i < str.size(); ++i)
        if ((uint32_t)(str[i] >> nlow) == H) {
          if (first < 0) first = (int)i;
          ++cnt;
        }
      if (first < 0) first = 0;
      group.insert(group.end(), {first, cnt, (int)sorted.size(), (int)ks.size()});
      sorted.insert(sorted.end(), ks.begin(), ks.end());
      max_home = std::max(max_home, cnt);
      max_inter = std::max(max_inter, (int)ks.size());
    }
    if (dev::rdm_mfma_lds(P.c64, max_home, max_inter) > budget && h < N) continue;
    R.nlow = nlow;
    R.ngroups = (int)group.size() / 4;
    R.max_home = max_home;
    R.max_inter = max_inter;
    R.group = (int*)P.dalloc(std::max<size_t>(group.size(), 4) * 4);
    R.inter = (uint32_t*)P.dalloc(std::max<size_t>(sorted.size(), 1) * 4);
    if (!group.empty()) HIPCHK(hipMemcpy(R.group, group.data(), group.size() * 4, hipMemcpyHostToDevice));
    if (!sorted.empty()) HIPCHK(hipMemcpy(R.inter, sorted.data(), sorted.size() * 4, hipMemcpyHostToDevice));
    R.ready = true;
    return;
  }
}

void rdm_columns(ffx_plan_s& P, int cs, const void* lam, const void* psi, int64_t rows, int64_t cols,
                 double* part, hipStream_t s) {
  const auto& R = P.rdm_k[cs];
  dev::RdmMfmaDev d{};
  d.lam = lam;
  d.psi = psi;
  d.rows = rows;
  d.cols = cols;
  d.norb = P.norb;
  d.nlow = R.nlow;
  d.ngroups = R.ngroups;
  d.max_home = R.max_home;
  d.max_inter = R.max_inter;
  d.group = R.group;
  d.inter = R.inter;
  d.rank_lo = P.rank_lo;
  d.rank_hi = P.rank_hi;
  d.part = part;
  dev::rdm_mfma(P.c64, d, s);
}

void transition_rdm(ffx_plan_s& P, const void* lam, const void* psi, void* lamT, void* psiT, double* part,
                    double* Tout, hipStream_t s) {
  const int N = P.norb, NN = N * N;
  if (N <= 16 && !P.rdm_pairs) {
    // column spin of each layout through the strings of one electron fewer, on
    // the matrix cores: beta on the alpha-major states, alpha on their transposes
    ensure_rank_tables(P);
    ensure_rdm_strings(P, 0);
    ensure_rdm_strings(P, 1);
    rdm_columns(P, 1, lam, psi, P.dim[0], P.dim[1], part, s);
    dev::rdm_reduce(part, P.dim[0], N, Tout + 2 * NN, s);
    dev::transpose(P.c64, psi, psiT, P.dim[0], P.dim[1], s);
    dev::transpose(P.c64, lam, lamT, P.dim[0], P.dim[1], s);
    rdm_columns(P, 0, lamT, psiT, P.dim[1], P.dim[0], part, s);
    dev::rdm_reduce(part, P.dim[1], N, Tout, s);
    check_launch();
    return;
  }
  // row spin of each layout from row pairs
  dev::rdm_rows(P.c64, lam, psi, P.dim[0], P.dim[1], P.d_masks[0], N, part, s);
  dev::rdm_reduce(part, P.dim[0], N, Tout, s);
  dev::transpose(P.c64, psi, psiT, P.dim[0], P.dim[1], s);
  dev::transpose(P.c64, lam, lamT, P.dim[0], P.dim[1], s);
  dev::rdm_rows(P.c64, lamT, psiT, P.dim[1], P.dim[0], P.d_masks[1], N, part, s);
  dev::rdm_reduce(part, P.dim[1], N, Tout + 2 * NN, s);
  check_launch();
}

}  // namespace

// ---------------------------------------------------------------------------
// exported API
// ---------------------------------------------------------------------------
extern "C" {

const char* ffx_last_error(void) { return ffx::last_error().c_str(); }

int64_t ffx_dim(int norb, int n) {
  if (norb < 1 || norb > 32 || n < 0 || n > norb) return -1;
  return binom(norb, n);
}

int ffx_strings(int norb, int n, uint64_t* out) {
  return guard([&] {
    if (ffx_dim(norb, n) < 0 || !out) throw Error(FFX_EINVAL, "bad norb/n or null output");
    auto s = make_strings(norb, n);
    std::copy(s.begin(), s.end(), out);
  });
}

int ffx_givens_decomposition(int norb, const double* U, int* p, double* c, double* s, double* phase) {
  return guard([&] {
    if (norb < 1 || norb > 32 || !U || !p || !c || !s || !phase) throw Error(FFX_EINVAL, "bad argument");
    if (!all_finite(U, (size_t)2 * norb * norb)) throw Error(FFX_EINVAL, "non-finite U");
    auto Um = load_complex(norb, U);
    Decomposition d = givens_decompose(norb, Um.data());
    for (size_t k = 0; k < d.rots.size(); ++k) {
      p[k] = d.rots[k].p;
      c[k] = d.rots[k].c;
      s[2 * k] = d.rots[k].s.real();
      s[2 * k + 1] = d.rots[k].s.imag();
    }
    for (int q = 0; q < norb; ++q) phase[q] = d.phase[q];
  });
}

int ffx_plan_create(ffx_plan* out, int norb, int na, int nb, ffx_dtype dtype, int device) {
  return guard([&] {
    if (!out) throw Error(FFX_EINVAL, "null output");
    *out = nullptr;
    if (norb < 1 || norb > 32 || na < 0 || na > norb || nb < 0 || nb > norb)
      throw Error(FFX_EINVAL, "norb must be in [1, 32] and 0 <= n_sigma <= norb");
    if (dtype != FFX_C128 && dtype != FFX_C64) throw Error(FFX_EINVAL, "unknown dtype");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw Error(FFX_EINVAL, "no such device");
    DeviceGuard dg(device);
    // the allocation-free sampler's device scratch: its address on this device
    double* scr = nullptr;
    HIPCHK(dev::sample_scratch(device, &scr));
    auto P = std::make_unique<ffx_plan_s>();
    P->norb = norb;
    P->n[0] = na;
    P->n[1] = nb;
    P->c64 = dtype == FFX_C64;
    P->device = device;
    for (int s = 0; s < 2; ++s) {
      P->str[s] = make_strings(norb, P->n[s]);
      P->dim[s] = (int64_t)P->str[s].size();
      std::vector<uint32_t> m32(P->str[s].begin(), P->str[s].end());
      P->d_masks[s] = (uint32_t*)P->dalloc(m32.size() * 4);
      HIPCHK(hipMemcpy(P->d_masks[s], m32.data(), m32.size() * 4, hipMemcpyHostToDevice));
    }
    if (P->dim[0] * P->dim[1] > (int64_t)1 << 40) throw Error(FFX_EINVAL, "state too large");
    if (P->dim[0] >= (1LL << 31) || P->dim[1] >= (1LL << 31)) throw Error(FFX_EINVAL, "dimension too large");
    P->W = std::min(norb, dev::max_window(P->c64));
    if (const char* e = std::getenv("FFX_WINDOW")) {  // narrower windows, for experiments
      int w = std::atoi(e);
      if (w >= 1 && w < P->W) P->W = w;
    }
    for (int s = 0; s < 2; ++s) {
      for (int a = 0; a + P->W <= norb; ++a) {
        WindowTable t = build_window_table(P->str[s], norb, P->n[s], a, P->W);
        dev::WinDev wd{};
        int* tab = (int*)P->dalloc(t.tab.size() * 4);
        int* cm = (int*)P->dalloc(t.chunk_m.size() * 4);
        int* co = (int*)P->dalloc(t.chunk_off.size() * 4);
        int* cl = (int*)P->dalloc(t.cls.size() * 4);
        HIPCHK(hipMemcpy(tab, t.tab.data(), t.tab.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(cm, t.chunk_m.data(), t.chunk_m.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(co, t.chunk_off.data(), t.chunk_off.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(cl, t.cls.data(), t.cls.size() * 4, hipMemcpyHostToDevice));
        wd.tab = tab;
        wd.chunk_m = cm;
        wd.chunk_off = co;
        wd.cls = cl;
        wd.n_chunks = (int)t.chunk_m.size();
        wd.n_cls = (int)t.cls.size();
        wd.a = a;
        wd.w = P->W;
        P->win[s].push_back(wd);
      }
    }
    // upload ring
    P->slot_bytes = (size_t)4 << 20;
    if (fault_hit("alloc") ||
        hipHostMalloc((void**)&P->h_ring, P->slot_bytes * ffx_plan_s::kSlots, hipHostMallocDefault) != hipSuccess)
      throw Error(FFX_ENOMEM, "pinned host allocation failed");
    P->d_ring = (char*)P->dalloc(P->slot_bytes * ffx_plan_s::kSlots);
    for (auto& e : P->ev) {
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      HIPCHK(hipEventRecord(e, nullptr));
    }
    // scratch
    const int64_t dmax = std::max(P->dim[0], P->dim[1]);
    for (int s = 0; s < 2; ++s) P->phase_tab[s] = P->dalloc((size_t)P->dim[s] * P->elem());
    P->dA = (double*)P->dalloc((size_t)P->dim[0] * 8);
    P->dB = (double*)P->dalloc((size_t)P->dim[1] * 8);
    P->dV = (double*)P->dalloc((size_t)norb * P->dim[1] * 8);
    P->n_partials = std::max<int>(dev::diag_expect_partials(P->dim[0], P->dim[1]),
                                  2 * dev::inner_partials(P->dim[0] * P->dim[1]));
    P->partials = (double*)P->dalloc((size_t)P->n_partials * 8);
    P->results = (double*)P->dalloc((size_t)ffx_plan_s::kResults * 8);
    P->results_cap = ffx_plan_s::kResults;
    P->rowout = (double*)P->dalloc((size_t)dmax * 2 * norb * 8);
    P->arena_doubles = (size_t)ffx_plan_s::kArenaSlots * (size_t)(P->dim[0] + P->dim[1]);
    P->arena = (double*)P->dalloc(P->arena_doubles * 8);
    // segment passes: for each column spin, the widest segment window whose
    // segments fit in LDS together with the stage tables and the member
    // offset tables of every register window inside the segment
    const size_t lds_cap = 160 * 1024 - 64;
    int64_t max_elems = (int64_t)((lds_cap - dev::seg_pass_lds(P->c64, 0, 0)) / P->elem());
    // the row-pair transition one-body kernel (the path above 16 orbitals) at
    // any size, for tests
    P->rdm_pairs = std::getenv("FFX_RDM_PAIRS") != nullptr;
    // FFX_DENSE=0 keeps every orbital rotation on the Givens sweeps (as do the forced small segments of
    // FFX_SEG_MAX, whose purpose is to run those sweeps' crossing paths at small sizes)
    if (const char* e = std::getenv("FFX_DENSE")) P->dense_max_dim = std::atoll(e) > 0 ? std::atoll(e) : 0;
    if (std::getenv("FFX_SEG_MAX")) P->dense_max_dim = 0;
    if (P->c64 || P->n[0] > 8 || P->n[1] > 8) P->dense_max_dim = 0;
    if (const char* e = std::getenv("FFX_SEG_MAX")) {  // smaller segments, for tests
      int64_t v = std::atoll(e);
      if (v >= 1 && v < max_elems) max_elems = v;
    }
    // lanes per LDS access cycle for the class loads: 128 bytes per cycle
    int lds_group_bytes = 128;
    if (const char* e = std::getenv("FFX_LDS_GROUP_BYTES")) {  // tuning knob (0: address order)
      const int v = std::atoi(e);
      if (v >= 0 && v <= 1024) lds_group_bytes = v;
    }
    const int lds_group = lds_group_bytes / (int)P->elem();
    // pack runs of configurations that share their orbitals above the segment
    // window back to back into one segment while they fit (0: one run per
    // segment; for tests)
    // row planes for complex128 rows split into segments: FFX_PLANES=0 (off),
    // 768 (default; measured faster) or 512 threads per block
    int plane_threads = 768;
    if (const char* e = std::getenv("FFX_PLANES")) {
      const int v = std::atoi(e);
      plane_threads = (v == 768 || v == 512) ? v : 0;
    }
    if (std::getenv("FFX_SEG_MAX")) plane_threads = 0;
    // FFX_PLANE_SEG_MAX=<elements>: shorter plane segments (tests of the plane
    // passes on rows split into segments, at small sizes)
    int64_t plane_seg_max = (int64_t)1 << 30;
    bool plane_seg_forced = false;
    if (const char* e = std::getenv("FFX_PLANE_SEG_MAX")) {
      const int64_t v = std::atoll(e);
      if (v >= 1) {
        plane_seg_max = v;
        plane_seg_forced = true;
      }
    }
    // FFX_PLANES_ALL=1: plane sets also where whole rows fit in LDS (tests of the plane passes at small sizes)
    const bool planes_all = std::getenv("FFX_PLANES_ALL") != nullptr;
    const char* pack_env = std::getenv("FFX_SEG_PACK");
    const bool pack_ok = !(pack_env && std::atoi(pack_env) == 0);
    int max_rows_x_seg = 0;
    for (int s = 0; s < 2; ++s) {
      auto& ss = P->seg[s];
      const auto& strs = P->str[s];
      std::vector<std::pair<int, int>> segs;
      std::vector<std::vector<SegWindowTable>> tabs;
      bool packed = false;
      int wt = norb;
      for (; wt >= 0; --wt) {
        segs = segment_runs(strs, wt);
        int64_t longest = 0;
        for (const auto& r : segs) longest = std::max<int64_t>(longest, r.second);
        if (longest > max_elems) continue;
        // Runs are contiguous in colex order.  At low filling most runs are
        // short (a handful of configurations per occupation of the top
        // orbitals); a block per run would mostly idle through the stages, so
        // consecutive runs share a block when that saves a quarter of the blocks.
        packed = false;
        if (pack_ok) {
          // room for the member offset tables of every register window (nl1
          // is at most min(a, electrons) + 1; each table padded to 16 bytes)
          const int W0 = std::min(P->W, wt), nc = s == 0 ? na : nb;
          size_t mt_bound = 0;
          for (int a = 0; W0 >= 2 && a + W0 <= wt; ++a) {
            const size_t nl1 = (size_t)std::min(a, nc) + 1;
            mt_bound = (mt_bound + 3) & ~(size_t)3;
            mt_bound += (((size_t)(W0 + 1) * nl1 + 3) & ~(size_t)3);
            for (int m = 0; m <= W0; ++m) mt_bound += nl1 * (((size_t)binom(W0, m) + 3) & ~(size_t)3);
          }
          const size_t fixed = dev::seg_pass_lds(P->c64, 0, (int)mt_bound);
          const int64_t cap = fixed < lds_cap ? std::min<int64_t>(max_elems, (int64_t)((lds_cap - fixed) / P->elem())) : 0;
          std::vector<std::pair<int, int>> groups = pack_runs(segs, cap);
          if (groups.size() * 4 <= segs.size() * 3) {
            segs = std::move(groups);
            packed = true;
          }
        }
        const int Wseg = std::min(P->W, wt);
        tabs.assign(segs.size(), {});
        size_t need = 0;
        for (size_t g = 0; g < segs.size(); ++g) {
          std::vector<uint64_t> sub(strs.begin() + segs[g].first, strs.begin() + segs[g].first + segs[g].second);
          size_t mt = 0;
          for (int a = 0; Wseg >= 2 && a + Wseg <= wt; ++a) {
            tabs[g].push_back(build_seg_window(sub, wt, a, Wseg, lds_group));
            mt = ((mt + 3) & ~(size_t)3) + tabs[g].back().mt.size();
          }
          need = std::max(need, dev::seg_pass_lds(P->c64, segs[g].second, (int)mt));
        }
        if (need <= lds_cap) break;
      }
      if (wt < 0) throw Error(FFX_EUNSUPPORTED, "no segment window fits in LDS");
      ss.wt = wt;
      ss.Wseg = std::min(P->W, wt);
      ss.n_seg = (int)segs.size();
      ss.max_len = 0;
      ss.max_mt = 0;
      for (const auto& sg : segs) ss.max_len = std::max(ss.max_len, sg.second);
      ss.threads = ss.max_len >= 4096 ? 1024 : (ss.max_len >= 1024 ? 256 : 64);
      if (const char* e = std::getenv("FFX_SEG_THREADS")) {  // block size override, for tuning
        int v = std::atoi(e);
        if (v >= 64 && v <= 1024 && v % 64 == 0) ss.threads = v;
      }
      ss.threads = dev::seg_pass_threads(P->c64, ss.Wseg, ss.threads);
      std::vector<dev::SegDev> hsegs;
      for (size_t g = 0; g < segs.size(); ++g) {
        const auto& sg = segs[g];
        ss.max_len = std::max(ss.max_len, sg.second);
        std::vector<dev::SegWinDev> wins;
        std::vector<int> mt_all;
        for (SegWindowTable& t : tabs[g]) {
          balance_seg_window(t, ss.Wseg, ss.threads / 64);
          dev::SegWinDev wd{};
          while (mt_all.size() % 4) mt_all.push_back(0);
          wd.mt_off = (int)mt_all.size();
          const std::vector<int> packed = pack_class_codes(t, wd.mt_off);
          int* code = (int*)P->dalloc(std::max<size_t>(packed.size(), 1) * 4);
          int* cm = (int*)P->dalloc(std::max<size_t>(t.chunk_m.size(), 1) * 4);
          if (!packed.empty()) HIPCHK(hipMemcpy(code, packed.data(), packed.size() * 4, hipMemcpyHostToDevice));
          if (!t.chunk_m.empty()) HIPCHK(hipMemcpy(cm, t.chunk_m.data(), t.chunk_m.size() * 4, hipMemcpyHostToDevice));
          wd.code = code;
          wd.chunk_m = cm;
          wd.n_chunks = (int)t.chunk_m.size();
          wd.nl1 = t.nl1;
          mt_all.insert(mt_all.end(), t.mt.begin(), t.mt.end());
          wins.push_back(wd);
        }
        while (mt_all.size() % 4) mt_all.push_back(0);  // staged as int4 words
        ss.max_mt = std::max(ss.max_mt, (int)mt_all.size());
        auto* dw = (dev::SegWinDev*)P->dalloc(std::max<size_t>(wins.size(), 1) * sizeof(dev::SegWinDev));
        if (!wins.empty())
          HIPCHK(hipMemcpy(dw, wins.data(), wins.size() * sizeof(dev::SegWinDev), hipMemcpyHostToDevice));
        int* dmt = (int*)P->dalloc(std::max<size_t>(mt_all.size(), 1) * 4);
        if (!mt_all.empty()) HIPCHK(hipMemcpy(dmt, mt_all.data(), mt_all.size() * 4, hipMemcpyHostToDevice));
        hsegs.push_back(dev::SegDev{sg.first, sg.second, dw, dmt, (int)mt_all.size(), 0, 0, 0, 0, 0});
      }
      // partner ranges of the crossing rotation on (wt - 1, wt): a segment whose
      // high part H lacks wt pairs its strings holding wt - 1 (the last C(wt-1,
      // k-1) of its C(wt, k)) with the first C(wt-1, k-1) strings of segment
      // H + {wt}, which lack wt - 1; both ranges run in the colex order of the
      // remaining k - 1 low orbitals.  Packed segments leave that rotation to
      // the window passes.  Applying it at load pays when (wt - 1, wt) is the
      // only pair that crosses the segment window (wt = norb - 1): then no
      // window pass runs at all.  With more orbitals above the window, window
      // passes run anyway and take that pair's rotations with the others,
      // while each rotation applied at load would start one more segment pass
      // (at 18 orbitals: 96 segment passes per DF step instead of 58).
      // FFX_CROSS_AT_LOAD=1 applies it at load in every case (tests).
      const bool cross_at_load = wt == norb - 1 || std::getenv("FFX_CROSS_AT_LOAD") != nullptr;
      if (wt >= 1 && wt < norb && segs.size() > 1 && !packed && cross_at_load) {
        const auto cr = crossing_ranges(strs, segs, wt, s == 0 ? na : nb);
        for (size_t g = 0; g < segs.size(); ++g) {
          if (!cr[g].has) continue;
          dev::SegDev& d = hsegs[g];
          d.cross_role = cr[g].role;
          d.cross_lo = cr[g].lo;
          d.cross_cnt = cr[g].cnt;
          d.cross_peer = cr[g].peer;
          ss.cross = true;
        }
      }
      ss.d_segs = (dev::SegDev*)P->dalloc(hsegs.size() * sizeof(dev::SegDev));
      HIPCHK(hipMemcpy(ss.d_segs, hsegs.data(), hsegs.size() * sizeof(dev::SegDev), hipMemcpyHostToDevice));
      ss.lds = dev::seg_pass_lds(P->c64, ss.max_len, ss.max_mt);
      // rows of this column spin's layout times segments: one partial sum per block
      max_rows_x_seg = std::max<int>(max_rows_x_seg, (int)(P->dim[1 - s] * ss.n_seg));
      // complex128 rows split into segments: visits whose rotations are all
      // real hold the real parts of each row segment in LDS and the imaginary
      // parts in registers (row planes).  The plane segments are the runs of
      // strings that share the orbitals above the highest plane window whose
      // runs fit the plane kernel: the whole row where its real parts fit (no
      // rotation crosses a segment: one pass per visit); otherwise, as at 18
      // orbitals, runs twice as long as the segment set's, with the rotations
      // on the orbitals above the window left to whole-spin window passes.
      if (!P->c64 && (ss.wt < norb || planes_all) && plane_threads > 0) {
        const int64_t pmax = std::min<int64_t>(dev::seg_pass_plane_max_len(plane_threads), plane_seg_max);
        for (int wp = norb; wp >= 1; --wp) {
          const int Wp = std::min(P->W, wp);
          if (Wp < 4) break;
          std::vector<std::pair<int, int>> psegs = segment_runs(strs, wp);
          int64_t longest = 0;
          for (const auto& r : psegs) longest = std::max<int64_t>(longest, r.second);
          if (longest > pmax) continue;
          // split rows: only where the plane segments are longer than the
          // segment set's and not packed runs of a low filling (whose many
          // short runs would leave most blocks idle)
          if (wp < norb && !(plane_seg_forced || (!packed && wp > ss.wt))) break;
          if (psegs.size() > 1 && Wp != 6) break;  // (the split-row plane kernel is built for width 6)
          std::vector<std::vector<SegWindowTable>> ptabs(psegs.size());
          size_t mt_max = 0, n_tabs = 0;
          for (size_t g = 0; g < psegs.size(); ++g) {
            std::vector<uint64_t> sub(strs.begin() + psegs[g].first,
                                      strs.begin() + psegs[g].first + psegs[g].second);
            size_t mt = 0;
            for (int a = 0; a + Wp <= wp; ++a) {
              ptabs[g].push_back(build_seg_window(sub, wp, a, Wp, lds_group_bytes / 8));
              mt = ((mt + 3) & ~(size_t)3) + ptabs[g].back().mt.size();
            }
            mt_max = std::max(mt_max, mt);
            n_tabs = std::max(n_tabs, ptabs[g].size());
          }
          // the row area holds 8-byte parts: sized as a complex64 row
          const size_t need = dev::seg_pass_lds(true, (int)longest, (int)mt_max + 3 * (int)n_tabs + 4);
          if (need > lds_cap) continue;
          auto& pl = P->plane[s];
          pl.wt = wp;
          pl.Wseg = Wp;
          pl.n_seg = (int)psegs.size();
          pl.max_len = (int)longest;
          pl.threads = plane_threads;
          pl.cross = false;
          pl.max_mt = 0;
          std::vector<dev::SegDev> hsegs;
          for (size_t g = 0; g < psegs.size(); ++g) {
            std::vector<dev::SegWinDev> wins;
            std::vector<int> mt_all;
            for (SegWindowTable& t : ptabs[g]) {
              balance_seg_window(t, Wp, plane_threads / 64);
              dev::SegWinDev wd{};
              while (mt_all.size() % 4) mt_all.push_back(0);
              wd.mt_off = (int)mt_all.size();
              const std::vector<int> packed = pack_class_codes(t, wd.mt_off);
              int* code = (int*)P->dalloc(std::max<size_t>(packed.size(), 1) * 4);
              int* cm = (int*)P->dalloc(std::max<size_t>(t.chunk_m.size(), 1) * 4);
              if (!packed.empty())
                HIPCHK(hipMemcpy(code, packed.data(), packed.size() * 4, hipMemcpyHostToDevice));
              if (!t.chunk_m.empty())
                HIPCHK(hipMemcpy(cm, t.chunk_m.data(), t.chunk_m.size() * 4, hipMemcpyHostToDevice));
              wd.code = code;
              wd.chunk_m = cm;
              wd.n_chunks = (int)t.chunk_m.size();
              wd.nl1 = t.nl1;
              mt_all.insert(mt_all.end(), t.mt.begin(), t.mt.end());
              wins.push_back(wd);
            }
            while (mt_all.size() % 4) mt_all.push_back(0);
            pl.max_mt = std::max(pl.max_mt, (int)mt_all.size());
            auto* dw = (dev::SegWinDev*)P->dalloc(std::max<size_t>(wins.size(), 1) * sizeof(dev::SegWinDev));
            if (!wins.empty())
              HIPCHK(hipMemcpy(dw, wins.data(), wins.size() * sizeof(dev::SegWinDev), hipMemcpyHostToDevice));
            int* dmt = (int*)P->dalloc(std::max<size_t>(mt_all.size(), 1) * 4);
            if (!mt_all.empty()) HIPCHK(hipMemcpy(dmt, mt_all.data(), mt_all.size() * 4, hipMemcpyHostToDevice));
            hsegs.push_back(dev::SegDev{psegs[g].first, psegs[g].second, dw, dmt, (int)mt_all.size(), 0, 0, 0, 0, 0});
          }
          pl.d_segs = (dev::SegDev*)P->dalloc(hsegs.size() * sizeof(dev::SegDev));
          HIPCHK(hipMemcpy(pl.d_segs, hsegs.data(), hsegs.size() * sizeof(dev::SegDev), hipMemcpyHostToDevice));
          pl.lds = dev::seg_pass_lds(true, pl.max_len, pl.max_mt);
          if (pl.lds > lds_cap) {
            pl = ffx_plan_s::SegSet{};
          } else {
            max_rows_x_seg = std::max<int>(max_rows_x_seg, (int)(P->dim[1 - s] * pl.n_seg));
          }
          break;
        }
      }
    }
    if (max_rows_x_seg > P->n_partials) {
      P->n_partials = max_rows_x_seg;
      P->partials = (double*)P->dalloc((size_t)P->n_partials * 8);
    }
    HIPCHK(hipDeviceSynchronize());
    *out = P.release();
  });
}

int ffx_plan_destroy(ffx_plan plan) {
  return guard([&] {
    if (!plan) return;
    DeviceGuard dg(plan->device);
    (void)hipDeviceSynchronize();
    delete plan;
  });
}

int ffx_plan_info(ffx_plan plan, int64_t* da, int64_t* db, int64_t* bytes) {
  return guard([&] {
    validate_plan(plan);
    if (da) *da = plan->dim[0];
    if (db) *db = plan->dim[1];
    if (bytes) *bytes = (int64_t)plan->state_bytes();
  });
}

int ffx_plan_strings(ffx_plan plan, int spin, uint64_t* out) {
  return guard([&] {
    validate_plan(plan);
    if ((spin != 0 && spin != 1) || !out) throw Error(FFX_EINVAL, "bad spin or null output");
    DeviceGuard dg(plan->device);
    std::vector<uint32_t> m(plan->dim[spin]);
    HIPCHK(hipMemcpy(m.data(), plan->d_masks[spin], m.size() * 4, hipMemcpyDeviceToHost));
    std::copy(m.begin(), m.end(), out);
  });
}

namespace {
void rotate_dense(ffx_plan_s& P, void* vec, const double* U_a, const double* U_b, void* workspace, hipStream_t s);
void check_rotation_args(int N, const double* U_a, const double* U_b);
}  // namespace

int ffx_apply_orbital_rotation(ffx_plan plan, void* vec, const double* U_a, const double* U_b, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !U_a) throw Error(FFX_EINVAL, "null vec or U_a");
    const int N = plan->norb;
    if (!all_finite(U_a, (size_t)2 * N * N) || (U_b && !all_finite(U_b, (size_t)2 * N * N)))
      throw Error(FFX_EINVAL, "non-finite U");
    DeviceGuard dg(plan->device);
    hipStream_t s = as_stream(stream);
    if (plan->dim[0] <= plan->dense_max_dim && plan->dim[1] <= plan->dense_max_dim) {
      // small sector: the dense form is the faster one (measured)
      check_rotation_args(N, U_a, U_b);
      if (!plan->dense_ws) plan->dense_ws = plan->dalloc((size_t)ffx_workspace_bytes(plan, 3));
      rotate_dense(*plan, vec, U_a, U_b, plan->dense_ws, s);
      return;
    }
    auto Ua = load_complex(N, U_a);
    std::vector<cd> Ub;
    if (U_b) Ub = load_complex(N, U_b);
    DecompPool pool;
    const Decomposition* da = pool.add(N, Ua);
    const Decomposition* db = U_b ? pool.add(N, Ub) : da;
    Program pr;
    pr.rot(da, db);
    Upload up(plan, s);
    Compiled c = compile_program(*plan, up, pr, FINAL_STORE, s);
    up.commit();
    execute_program(*plan, c, vec, vec, nullptr, s);
  });
}

namespace {
// Gamma' = C_a Gamma C_b^T: compound matrices on the device, then two complex products on the FP64 matrix
// cores; workspace holds C_a, C_b and the intermediate (ffx_workspace_bytes(plan, 3))
void rotate_dense(ffx_plan_s& P, void* vec, const double* U_a, const double* U_b, void* workspace, hipStream_t s) {
  const int N = P.norb;
  const double* Ubp = U_b ? U_b : U_a;
  {
    const int64_t da = P.dim[0], db = P.dim[1];
    auto r256 = [](int64_t b) { return (b + 255) / 256 * 256; };
    char* ws = (char*)workspace;
    void* Ca = ws;
    void* Cb = ws + r256(da * da * 16);
    void* T = (char*)Cb + r256(db * db * 16);
    Upload up(&P, s);
    const double* dUa = up.put(U_a, (size_t)2 * N * N);
    const double* dUb = up.put(Ubp, (size_t)2 * N * N);
    up.commit();
    dev::compound_matrix(P.d_masks[0], da, P.n[0], N, dUa, Ca, s);
    dev::compound_matrix(P.d_masks[1], db, P.n[1], N, dUb, Cb, s);
    // T = Gamma C_b^T (element (k, n) of C_b^T is C_b[n][k]), then Gamma' = C_a T
    dev::zgemm_mfma(vec, db, Cb, 1, db, T, db, (int)da, (int)db, (int)db, s);
    dev::zgemm_mfma(Ca, da, T, db, 1, vec, db, (int)da, (int)db, (int)da, s);
    check_launch();
  }
}

void check_rotation_args(int N, const double* U_a, const double* U_b) {
  if (!all_finite(U_a, (size_t)2 * N * N) || (U_b && !all_finite(U_b, (size_t)2 * N * N)))
    throw Error(FFX_EINVAL, "non-finite U");
  for (const double* u : {U_a, U_b}) {
    if (!u) continue;
    auto Um = load_complex(N, u);
    if (unitarity_defect(N, Um.data()) > 1e-10) throw Error(FFX_ENOTUNITARY, "orbital rotation is not unitary");
  }
}
}  // namespace

int ffx_apply_orbital_rotation_dense(ffx_plan plan, void* vec, const double* U_a, const double* U_b, void* workspace,
                                     void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !U_a || !workspace) throw Error(FFX_EINVAL, "null vec, U_a or workspace");
    ffx_plan_s& P = *plan;
    if (P.c64) throw Error(FFX_EUNSUPPORTED, "the dense form is built for complex128 states");
    if (P.n[0] > 8 || P.n[1] > 8 || P.dim[0] > 4096 || P.dim[1] > 4096)
      throw Error(FFX_EUNSUPPORTED, "the dense form takes at most 8 electrons and 4096 configurations per spin");
    check_rotation_args(P.norb, U_a, U_b);
    DeviceGuard dg(P.device);
    rotate_dense(P, vec, U_a, U_b, workspace, as_stream(stream));
  });
}

namespace {
// script-U(B) [gate] script-U(B)^dag when a basis rotation B is given
struct BasisWrap {
  DecompPool pool;
  const Decomposition* to = nullptr;
  const Decomposition* from = nullptr;
  BasisWrap(int N, const double* B) {
    if (!B) return;
    if (!all_finite(B, (size_t)2 * N * N)) throw Error(FFX_EINVAL, "non-finite basis rotation");
    std::vector<cd> U = load_complex(N, B);
    from = pool.add(N, U);
    to = pool.add(N, dagger(N, U));
  }
  void before(Program& pr) const {
    if (to) pr.rot(to, to);
  }
  void after(Program& pr) const {
    if (from) pr.rot(from, from);
  }
};
}  // namespace

int ffx_apply_num_op_sum_evolution(ffx_plan plan, void* vec, const double* lam_a, const double* lam_b,
                                   double time, const double* basis_U, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !lam_a) throw Error(FFX_EINVAL, "null vec or lam_a");
    const int N = plan->norb;
    if (!std::isfinite(time) || !all_finite(lam_a, N) || (lam_b && !all_finite(lam_b, N)))
      throw Error(FFX_EINVAL, "non-finite parameter");
    BasisWrap bw(N, basis_U);
    DeviceGuard dg(plan->device);
    hipStream_t s = as_stream(stream);
    Program pr;
    DiagSpec d;
    d.lin_a = lam_a;
    d.lin_b = lam_b ? lam_b : lam_a;
    bw.before(pr);
    pr.phase(pr.add_diag(d), -time);
    bw.after(pr);
    Upload up(plan, s);
    Compiled c = compile_program(*plan, up, pr, FINAL_STORE, s);
    up.commit();
    execute_program(*plan, c, vec, vec, nullptr, s);
  });
}

int ffx_apply_diag_coulomb_evolution(ffx_plan plan, void* vec, const double* J_aa, const double* J_ab,
                                     const double* J_bb, double time, const double* basis_U, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !J_aa) throw Error(FFX_EINVAL, "null vec or J_aa");
    const int N = plan->norb;
    const double* Jab = J_ab ? J_ab : J_aa;
    const double* Jbb = J_bb ? J_bb : J_aa;
    if (!std::isfinite(time) || !all_finite(J_aa, (size_t)N * N) || !all_finite(Jab, (size_t)N * N) ||
        !all_finite(Jbb, (size_t)N * N))
      throw Error(FFX_EINVAL, "non-finite parameter");
    BasisWrap bw(N, basis_U);
    DeviceGuard dg(plan->device);
    hipStream_t s = as_stream(stream);
    Program pr;
    DiagSpec d;
    d.Qa = J_aa;
    d.Qb = Jbb;
    d.C = Jab;
    bw.before(pr);
    pr.phase(pr.add_diag(d), -time);
    bw.after(pr);
    Upload up(plan, s);
    Compiled c = compile_program(*plan, up, pr, FINAL_STORE, s);
    up.commit();
    execute_program(*plan, c, vec, vec, nullptr, s);
  });
}

namespace {

// Q(tau) = exp(-i tau h) = V diag(exp(-i eps tau)) V^dag: the one-body factor as an orbital rotation
std::vector<cd> one_body_rotation(const DFHost& df, int N, double tau) {
  std::vector<cd> Q((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      cd acc = 0.0;
      for (int k = 0; k < N; ++k) acc += df.V[i * N + k] * std::exp(cd(0.0, -df.eps[k] * tau)) * std::conj(df.V[j * N + k]);
      Q[i * N + j] = acc;
    }
  return Q;
}

// A product formula, given as its merged list of (term, time), as one gate
// program.  The state is kept in the basis of the last two-body term visited:
// psi = script-U(B) phi.  A one-body factor exp(-i tau sum h a+ a) is the
// orbital rotation Q(tau) (Table 1: quadratic Hamiltonian evolution), so it
// only updates B <- Q B and is carried into the next change of basis,
// script-U(U_t^dag B).  A step thus costs one orbital rotation per two-body
// term plus the final return to the orbital basis, and the one-body term adds
// none.
Program product_formula_program(const DFHost& df, int N, const std::vector<std::pair<int, double>>& m,
                                DecompPool& pool) {
  std::map<std::pair<int, int>, const Decomposition*> rot_cache;
  Program pr;
  std::vector<int> weight((size_t)df.L + 1, -1);
  for (int t = 1; t <= df.L; ++t) weight[t] = pr.add_diag(df_weight_spec(df, t));
  std::vector<cd> B((size_t)N * N, 0.0);  // basis of the stored vector, with the pending one-body factors
  for (int i = 0; i < N; ++i) B[i * N + i] = 1.0;
  int basis = -1;        // two-body term whose basis B started from (-1: the orbital basis)
  bool pending = false;  // B carries one-body factors since that change of basis
  for (auto& e : m) {
    if (e.first == 0) {
      B = matmul(N, one_body_rotation(df, N, e.second), B);
      pending = true;
      continue;
    }
    const Decomposition* d;
    auto key = std::make_pair(basis, e.first);
    auto it = rot_cache.find(key);
    if (!pending && it != rot_cache.end()) {
      d = it->second;
    } else {
      d = pool.add(N, matmul(N, dagger(N, df.Wm(e.first)), B));
      if (!pending) rot_cache.emplace(key, d);
    }
    pr.rot(d, d);
    pr.phase(weight[e.first], -e.second);
    B = df.Wm(e.first);
    basis = e.first;
    pending = false;
  }
  const Decomposition* d = pool.add(N, B);
  pr.rot(d, d);
  return pr;
}

}  // namespace

int ffx_apply_df_trotter_step(ffx_plan plan, void* vec, const ffx_df_ham* ham, double dt, int n_steps,
                              int order, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec) throw Error(FFX_EINVAL, "null vec");
    if (n_steps < 0 || order < 0 || order > 8 || !std::isfinite(dt)) throw Error(FFX_EINVAL, "bad n_steps/order/dt");
    ffx_plan_s& P = *plan;
    const int N = P.norb;
    DFHost df = load_df(P, ham);
    if (n_steps == 0) return;
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    std::vector<std::pair<int, double>> seq;
    for (int r = 0; r < n_steps; ++r) product_formula(order, dt, df.L + 1, seq);
    // merge equal neighbours: D(t1) D(t2) = D(t1 + t2) with no rotation between
    std::vector<std::pair<int, double>> m;
    for (auto& e : seq) {
      if (!m.empty() && m.back().first == e.first)
        m.back().second += e.second;
      else
        m.push_back(e);
    }
    DecompPool pool;
    Program pr = product_formula_program(df, N, m, pool);
    Upload up(&P, s);
    Compiled c = compile_program(P, up, pr, FINAL_STORE, s);
    up.commit();
    execute_program(P, c, vec, vec, nullptr, s);
  });
}

int ffx_simulate_trotter_diag_coulomb(ffx_plan plan, void* vec, const double* h, const double* J_aa,
                                      const double* J_ab, const double* J_bb, double dt, int n_steps, int order,
                                      void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !h || !J_aa) throw Error(FFX_EINVAL, "null vec, h or J_aa");
    if (n_steps < 0 || order < 0 || order > 8 || !std::isfinite(dt)) throw Error(FFX_EINVAL, "bad n_steps/order/dt");
    ffx_plan_s& P = *plan;
    const int N = P.norb;
    const double* Jab = J_ab ? J_ab : J_aa;
    const double* Jbb = J_bb ? J_bb : J_aa;
    if (!all_finite(h, (size_t)N * N) || !all_finite(J_aa, (size_t)N * N) || !all_finite(Jab, (size_t)N * N) ||
        !all_finite(Jbb, (size_t)N * N))
      throw Error(FFX_EINVAL, "non-finite parameter");
    for (int p = 0; p < N; ++p)
      for (int q = 0; q < p; ++q)
        if (std::abs(h[p * N + q] - h[q * N + p]) > 1e-12 * std::max(1.0, std::abs(h[p * N + q])))
          throw Error(FFX_EINVAL, "h is not symmetric");
    // the one-body term's eigenbasis (the two-body term is already diagonal)
    const ffx_df_ham one{N, 0, h, nullptr, nullptr};
    DFHost df = load_df(P, &one);
    if (n_steps == 0) return;
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    // term 0 = the one-body term (applied first), term 1 = the diagonal Coulomb term
    std::vector<std::pair<int, double>> seq;
    for (int r = 0; r < n_steps; ++r) product_formula(order, dt, 2, seq);
    std::vector<std::pair<int, double>> m;
    for (auto& e : seq) {
      if (!m.empty() && m.back().first == e.first)
        m.back().second += e.second;
      else
        m.push_back(e);
    }
    // exp(-i tau H_1) is the orbital rotation Q(tau) = exp(-i tau h); consecutive one-body factors
    // collect into one rotation B, applied before the next diagonal Coulomb evolution
    DecompPool pool;
    Program pr;
    DiagSpec dc;
    dc.Qa = J_aa;
    dc.Qb = Jbb;
    dc.C = Jab;
    const int w = pr.add_diag(dc);
    std::vector<cd> B;
    for (auto& e : m) {
      if (e.first == 0) {
        const std::vector<cd> Q = one_body_rotation(df, N, e.second);
        B = B.empty() ? Q : matmul(N, Q, B);
        continue;
      }
      if (!B.empty()) {
        const Decomposition* d = pool.add(N, B);
        pr.rot(d, d);
        B.clear();
      }
      pr.phase(w, -e.second);
    }
    if (!B.empty()) {
      const Decomposition* d = pool.add(N, B);
      pr.rot(d, d);
    }
    Upload up(&P, s);
    Compiled c = compile_program(P, up, pr, FINAL_STORE, s);
    up.commit();
    execute_program(P, c, vec, vec, nullptr, s);
  });
}

int ffx_lucj_n_params(int norb, int n_reps) {
  if (norb < 1 || n_reps < 0) return -1;
  return n_reps * (2 * norb * norb + 2 * norb - 1);
}

int ffx_apply_lucj(ffx_plan plan, void* vec, const ffx_lucj* op, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec) throw Error(FFX_EINVAL, "null vec");
    ffx_plan_s& P = *plan;
    LUCJHost L = load_lucj(P, op);
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    DecompPool pool;
    LUCJParts g = lucj_parts(P, L, pool, false);
    Program pr = lucj_forward_program(g, L.R);
    Upload up(&P, s);
    const double* a = up.put((const double*)g.a.data(), 2 * g.a.size());
    const double* b = up.put((const double*)g.b.data(), 2 * g.b.size());
    Compiled c = compile_program(P, up, pr, FINAL_STORE, s);
    up.commit();
    dev::outer(P.c64, a, b, vec, P.dim[0], P.dim[1], s);
    check_launch();
    execute_program(P, c, vec, vec, nullptr, s);
  });
}

int64_t ffx_workspace_bytes(ffx_plan plan, int what) {
  if (!plan) return -1;
  const int64_t S = ((int64_t)plan->state_bytes() + 255) / 256 * 256;
  if (what == 0) return S;
  if (what == 2) return 4 * S;
  if (what == 3) {
    auto r256 = [](int64_t b) { return (b + 255) / 256 * 256; };
    return r256(plan->dim[0] * plan->dim[0] * 16) + r256(plan->dim[1] * plan->dim[1] * 16) +
           r256(plan->dim[0] * plan->dim[1] * 16);
  }
  const int64_t dmax = std::max(plan->dim[0], plan->dim[1]);
  const int64_t part = ((int64_t)plan->norb * plan->norb * dmax * 16 + 255) / 256 * 256;
  return 5 * S + part;
}

int ffx_df_energy(ffx_plan plan, const void* vec, const ffx_df_ham* ham, double* energy, void* workspace,
                  void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !energy || !workspace) throw Error(FFX_EINVAL, "null pointer");
    ffx_plan_s& P = *plan;
    const int N = P.norb;
    DFHost df = load_df(P, ham);
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    void* tmp = workspace;
    DecompPool pool;
    std::vector<Program> progs(df.L + 1);
    for (int t = 0; t <= df.L; ++t) {
      const Decomposition* d = pool.add(N, dagger(N, df.Wm(t)));
      progs[t].rot(d, d);
      progs[t].reduce(progs[t].add_diag(df_weight_spec(df, t)), P.results + t);
    }
    Upload up(&P, s);
    std::vector<Compiled> cs;
    for (auto& pr : progs) cs.push_back(compile_program(P, up, pr, FINAL_NONE, s));
    up.commit();
    for (auto& c : cs) execute_program(P, c, vec, tmp, nullptr, s);
    std::vector<double> r(df.L + 1);
    HIPCHK(hipMemcpyAsync(r.data(), P.results, r.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double e = 0;
    for (double x : r) e += x;
    *energy = e;
  });
}

namespace {

// H psi for a DF Hamiltonian.  The one-body term goes either through the
// eigenbasis of h (two orbital rotations around a diagonal scale, a gate
// program like the two-body terms) or directly, as sum_pq h_pq E_pq applied by
// rows of each spin from a sparse table (the beta spin on the transposed
// state).  Direct is taken when the tables are short (sparse h or few
// electrons): at most 48 entries per configuration over both spins.
struct HamAction {
  std::vector<Compiled> cs;  // gate programs: the two-body terms, after the one-body term when it is one
  bool direct = false;
  struct Tab {
    int64_t* off = nullptr;
    int32_t* src = nullptr;
    double* coef = nullptr;
  } tab[2];
  // two-body terms whose basis is exactly the identity (a diagonal Coulomb
  // Hamiltonian's term) ride along in the direct alpha pass as a diagonal
  dev::OneBodyDiag diag{nullptr, nullptr, nullptr, nullptr, 0};
  std::vector<void*> bufs;
  HamAction() = default;
  HamAction(const HamAction&) = delete;
  HamAction& operator=(const HamAction&) = delete;
  ~HamAction() {
    for (void* b : bufs) (void)hipFree(b);  // hipFree waits for the device
  }
  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (fault_hit("alloc") || hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess)
      throw Error(FFX_ENOMEM, "device allocation failed");
    bufs.push_back(p);
    return p;
  }
};

// Chooses the route of the one-body term (A.direct) and, for the direct route,
// builds its tables on the device.
void prepare_one_body(ffx_plan_s& P, const double* h, HamAction& A) {
  const int N = P.norb;
  std::vector<double> hv(h, h + (size_t)N * N);
  OneBodyTable t[2];
  bool direct = false;
  const char* mode = std::getenv("FFX_ONEBODY");  // "direct" / "rot": force a path (tests)
  if (mode && std::string(mode) == "rot") {
    direct = false;
  } else {
    const bool forced = mode && std::string(mode) == "direct";
    // expected entries per configuration from the off-diagonal nonzeros of h (a configuration with n
    // electrons reaches a given q outside it from each occupied p with probability (N - n) / (N - 1))
    double offdiag = 0;
    for (int p = 0; p < N; ++p)
      for (int q = 0; q < N; ++q)
        if (p != q && hv[(size_t)p * N + q] != 0.0) offdiag += 1.0;
    double est = 0;
    for (int sp = 0; sp < 2; ++sp)
      est += 1.0 + (N > 1 ? P.n[sp] * (offdiag / N) * (double)(N - P.n[sp]) / (N - 1) : 0.0);
    if (forced || est <= 64.0) {
      for (int sp = 0; sp < 2; ++sp) t[sp] = build_one_body_table(N, P.str[sp], hv);
      const double per = (double)t[0].src.size() / (double)P.dim[0] + (double)t[1].src.size() / (double)P.dim[1];
      direct = forced || per <= 48.0;
    }
  }
  A.direct = direct;
  if (!direct) return;
  for (int sp = 0; sp < 2; ++sp) {
    HamAction::Tab& d = A.tab[sp];
    d.off = (int64_t*)A.alloc(t[sp].off.size() * 8);
    d.src = (int32_t*)A.alloc(t[sp].src.size() * 4);
    d.coef = (double*)A.alloc(t[sp].coef.size() * 8);
    HIPCHK(hipMemcpy(d.off, t[sp].off.data(), t[sp].off.size() * 8, hipMemcpyHostToDevice));
    if (!t[sp].src.empty()) {
      HIPCHK(hipMemcpy(d.src, t[sp].src.data(), t[sp].src.size() * 4, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(d.coef, t[sp].coef.data(), t[sp].coef.size() * 8, hipMemcpyHostToDevice));
    }
  }
}

void build_ham_action(ffx_plan_s& P, const DFHost& df, const double* h, DecompPool& pool, hipStream_t s,
                      HamAction& A) {
  const int N = P.norb;
  prepare_one_body(P, h, A);
  // with the direct route, the terms in the orbital basis join its alpha pass
  std::vector<char> folded((size_t)df.L + 1, 0);
  if (A.direct) {
    std::vector<double> Jsum((size_t)N * N, 0.0);
    bool any = false;
    for (int t = 1; t <= df.L; ++t) {
      bool ident = true;
      for (int i = 0; i < N && ident; ++i)
        for (int j = 0; j < N; ++j)
          if (df.U[t - 1][i * N + j] != (i == j ? cd(1.0, 0.0) : cd(0.0, 0.0))) {
            ident = false;
            break;
          }
      if (!ident) continue;
      folded[t] = 1;
      any = true;
      for (int i = 0; i < N * N; ++i) Jsum[i] += df.J[t - 1][i];
    }
    if (any) {
      // weight 1/2 (x_a + x_b)^T J (x_a + x_b) as per-string tables A, B and the cross table V
      double* dJ = (double*)A.alloc((size_t)N * N * 8);
      HIPCHK(hipMemcpy(dJ, Jsum.data(), (size_t)N * N * 8, hipMemcpyHostToDevice));
      double* tA = (double*)A.alloc((size_t)P.dim[0] * 8);
      double* tB = (double*)A.alloc((size_t)P.dim[1] * 8);
      double* tV = (double*)A.alloc((size_t)N * P.dim[1] * 8);
      dev::DiagSpecDev spec{nullptr, nullptr, dJ, dJ, dJ};
      dev::diag_tables(P.d_masks[0], P.dim[0], P.d_masks[1], P.dim[1], N, spec, tA, tB, tV, s);
      check_launch();
      A.diag = dev::OneBodyDiag{tA, tB, tV, P.d_masks[0], N};
    }
  }
  std::vector<Program> terms = df_term_programs(df, pool, N);
  Upload up(&P, s);
  for (int term = A.direct ? 1 : 0; term <= df.L; ++term)
    if (!folded[term]) A.cs.push_back(compile_program(P, up, terms[term], term == 0 ? FINAL_STORE : FINAL_ACCUM, s));
  up.commit();
}

// out = sum_pq h_pq E_pq in from the direct tables; tmp is a state-sized work buffer; in, out, tmp distinct
void apply_one_body_direct(ffx_plan_s& P, const HamAction& A, const void* in, void* out, void* tmp,
                           hipStream_t s) {
  const int64_t da = P.dim[0], db = P.dim[1];
  // beta: on the transposed state, rows = beta configurations
  dev::transpose(P.c64, in, tmp, da, db, s);
  check_launch();
  const dev::OneBodyDiag none{nullptr, nullptr, nullptr, nullptr, 0};
  dev::onebody_rows(P.c64, tmp, out, nullptr, db, da, A.tab[1].off, A.tab[1].src, A.tab[1].coef, none, s);
  check_launch();
  dev::transpose(P.c64, out, tmp, db, da, s);
  check_launch();
  // alpha, plus the beta part
  dev::onebody_rows(P.c64, in, out, tmp, da, db, A.tab[0].off, A.tab[0].src, A.tab[0].coef, A.diag, s);
  check_launch();
}

// out = H in; tmp is a state-sized work buffer.  in, out and tmp are distinct.
void apply_ham(ffx_plan_s& P, const HamAction& A, const void* in, void* out, void* tmp, hipStream_t s) {
  size_t k = 0;
  if (A.direct) {
    apply_one_body_direct(P, A, in, out, tmp, s);
  } else {
    execute_program(P, A.cs[k++], in, out, nullptr, s);
  }
  for (; k < A.cs.size(); ++k) execute_program(P, A.cs[k], in, tmp, out, s);
}

}  // namespace

int ffx_apply_df_hamiltonian(ffx_plan plan, const void* vec, void* out, const ffx_df_ham* ham, void* workspace,
                             void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !out || !workspace) throw Error(FFX_EINVAL, "null pointer");
    if (vec == out || vec == workspace || out == workspace)
      throw Error(FFX_EINVAL, "vec, out and workspace must be distinct buffers");
    ffx_plan_s& P = *plan;
    DFHost df = load_df(P, ham);
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    DecompPool pool;
    HamAction A;
    build_ham_action(P, df, ham->h, pool, s, A);
    apply_ham(P, A, vec, out, workspace, s);
  });
}

int ffx_df_evolve_exact(ffx_plan plan, void* vec, const ffx_df_ham* ham, double time, double tol, void* workspace,
                        int* n_matvec, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !workspace) throw Error(FFX_EINVAL, "null pointer");
    if (!std::isfinite(time) || !(tol > 0.0) || !std::isfinite(tol)) throw Error(FFX_EINVAL, "bad time or tolerance");
    ffx_plan_s& P = *plan;
    DFHost df = load_df(P, ham);
    double lo, hi;
    df_spectrum_bounds(df, P.norb, P.n[0], P.n[1], &lo, &hi);
    const double c = 0.5 * (lo + hi);
    // a little room so that rounding in the bounds cannot leave an eigenvalue outside
    const double r = 0.5 * (hi - lo) * (1.0 + 1e-9) + 1e-12 * std::max(1.0, std::abs(c));
    const double z = r * std::abs(time);
    const double kmax_d = std::ceil(z + 10.0 * std::cbrt(z) + 60.0);
    if (kmax_d > 1e6) throw Error(FFX_EUNSUPPORTED, "evolution time too long for one expansion");
    const int kmax = (int)kmax_d;
    const std::vector<double> J = bessel_j_series(z, kmax);
    // truncation: the dropped terms weigh 2 sum_{j > K} |J_j(z)| at most (each
    // T_j of the shifted and scaled H has norm <= 1)
    int K = kmax;
    {
      double tail = 0.0;
      for (int k = kmax; k >= 1; --k) {
        if (tail + 2.0 * std::abs(J[k]) > 0.5 * tol) break;
        tail += 2.0 * std::abs(J[k]);
        K = k - 1;
      }
    }
    if (K == kmax) throw Error(FFX_EUNSUPPORTED, "Chebyshev expansion did not converge within its length");
    // coefficient of T_k: (2 - delta_k0) (-i)^k J_k(r time) exp(-i c time)
    auto coef = [&](int k) {
      double jk = J[k] * ((time < 0 && (k & 1)) ? -1.0 : 1.0);
      cd ipow = (k % 4 == 0) ? cd(1, 0) : (k % 4 == 1) ? cd(0, -1) : (k % 4 == 2) ? cd(-1, 0) : cd(0, 1);
      return (k == 0 ? 1.0 : 2.0) * jk * ipow * std::exp(cd(0.0, -c * time));
    };
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    DecompPool pool;
    HamAction A;
    build_ham_action(P, df, ham->h, pool, s, A);
    const size_t S = P.state_bytes();
    const size_t Sa = (S + 255) / 256 * 256;
    char* ws = (char*)workspace;
    void* tprev = ws;
    void* tcur = ws + Sa;
    void* y = ws + 2 * Sa;
    void* tmp = ws + 3 * Sa;
    const int64_t n = P.elems();
    HIPCHK(hipMemcpyAsync(tprev, vec, S, hipMemcpyDeviceToDevice, s));  // T_0 = vec
    const cd c0 = coef(0);
    dev::zscale(P.c64, vec, n, c0.real(), c0.imag(), s);
    check_launch();
    for (int k = 1; k <= K; ++k) {
      // k = 1: T_1 = (H - c) T_0 / r into tcur; k >= 2: T_k = 2 (H - c) T_{k-1} / r - T_{k-2}
      const void* src = k == 1 ? tprev : tcur;
      apply_ham(P, A, src, y, tmp, s);
      const cd ck = coef(k);
      if (k == 1) {
        dev::cheb_step(P.c64, y, tprev, tcur, vec, n, 1.0 / r, -c / r, 0.0, ck.real(), ck.imag(), s);
      } else {
        dev::cheb_step(P.c64, y, tcur, tprev, vec, n, 2.0 / r, -2.0 * c / r, -1.0, ck.real(), ck.imag(), s);
        std::swap(tprev, tcur);
      }
      check_launch();
    }
    if (n_matvec) *n_matvec = K;
  });
}

int ffx_state_distance(ffx_plan plan, const void* x, const void* y, double* dist, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!x || !y || !dist) throw Error(FFX_EINVAL, "null pointer");
    ffx_plan_s& P = *plan;
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    dev::dist2(P.c64, x, y, P.elems(), P.partials, P.results, s);
    check_launch();
    double d2 = 0;
    HIPCHK(hipMemcpyAsync(&d2, P.results, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *dist = std::sqrt(d2);
  });
}

int ffx_lucj_energy_grad(ffx_plan plan, const ffx_lucj* op, const ffx_df_ham* ham, double* energy, double* grad,
                         void* psi_out, void* workspace, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!energy || !grad || !workspace) throw Error(FFX_EINVAL, "null pointer");
    ffx_plan_s& P = *plan;
    const int N = P.norb;
    std::unique_ptr<LUCJGrad> G = build_lucj_grad(P, op, ham);
    const int R = G->L.R;
    const int Lt = G->df.L;
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    // result block: energy, per repetition the transition matrices and the diagonal-gate gradients
    P.results_for(16 + (size_t)R * (8 * (size_t)N * N + 2 * N), s);
    const size_t S = P.state_bytes();
    const size_t Sa = (S + 255) / 256 * 256;
    char* ws = (char*)workspace;
    void* lam = ws;
    void* tmp = ws + Sa;
    void* psiT = ws + 2 * Sa;
    void* lamT = ws + 3 * Sa;
    void* psi = ws + 4 * Sa;  // the reverse sweep uncomputes it; psi_out gets a copy
    double* part = (double*)(ws + 5 * Sa);
    HamAction onebody;
    prepare_one_body(P, ham->h, onebody);
    Upload up(&P, s);
    const double* sa = up.put((const double*)G->g.a.data(), 2 * G->g.a.size());
    const double* sb = up.put((const double*)G->g.b.data(), 2 * G->g.b.size());
    Compiled c_fwd = compile_program(P, up, G->fwd, FINAL_STORE, s);
    std::vector<Compiled> c_terms, c_urot, c_udiag;
    for (int t = 0; t <= Lt; ++t)
      c_terms.push_back(compile_program(P, up, G->terms[t], t == 0 ? FINAL_STORE : FINAL_ACCUM, s));
    for (int k = 0; k < R; ++k) {
      c_urot.push_back(compile_program(P, up, G->undo_rot[k], FINAL_STORE, s));
      c_udiag.push_back(compile_program(P, up, G->undo_diag[k], FINAL_STORE, s));
    }
    up.commit();
    // forward
    dev::outer(P.c64, sa, sb, psi, P.dim[0], P.dim[1], s);
    check_launch();
    execute_program(P, c_fwd, psi, psi, nullptr, s);
    if (psi_out) HIPCHK(hipMemcpyAsync(psi_out, psi, S, hipMemcpyDeviceToDevice, s));
    // costate lambda = H psi (the one-body term directly from its tables when they are short)
    for (int t = 0; t <= Lt; ++t) {
      if (t == 0 && onebody.direct)
        apply_one_body_direct(P, onebody, psi, lam, tmp, s);
      else if (t == 0)
        execute_program(P, c_terms[t], psi, lam, nullptr, s);
      else
        execute_program(P, c_terms[t], psi, tmp, lam, s);
    }
    // energy <psi|lambda>
    dev::inner(P.c64, psi, lam, P.elems(), P.partials, P.results, s);
    check_launch();
    // reverse sweep: uncompute psi and lambda, collecting transition matrices
    const int NN = N * N;
    double* Tdev = P.results + 16;                     // per rep: T_b (alpha, beta), T_a (alpha, beta)
    double* Ddev = P.results + 16 + (size_t)R * 8 * NN;  // per rep: 2N-1 diagonal-gate gradients
    auto rdm = [&](double* Tout) { transition_rdm(P, lam, psi, lamT, psiT, part, Tout, s); };
    for (int k = R - 1; k >= 0; --k) {
      execute_program(P, c_urot[k], psi, psi, nullptr, s);
      execute_program(P, c_urot[k], lam, lam, nullptr, s);
      rdm(Tdev + (size_t)k * 8 * NN);
      dev::diag_grad_rows(P.c64, lam, psi, P.dim[0], P.dim[1], P.d_masks[1], N, P.rowout, s);
      dev::diag_grad_combine(P.rowout, P.dim[0], P.d_masks[0], N, Ddev + (size_t)k * (2 * N), s);
      check_launch();
      execute_program(P, c_udiag[k], psi, psi, nullptr, s);
      execute_program(P, c_udiag[k], lam, lam, nullptr, s);
      rdm(Tdev + (size_t)k * 8 * NN + 4 * NN);
    }
    std::vector<double> res(16 + (size_t)R * (8 * NN + 2 * N));
    HIPCHK(hipMemcpyAsync(res.data(), P.results, res.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *energy = res[0];
    // both spins summed: T = T_alpha + T_beta
    std::vector<std::vector<double>> tb(R), ta(R);
    std::vector<const double*> Tb(R), Ta(R), D(R);
    for (int k = 0; k < R; ++k) {
      const double* b = res.data() + 16 + (size_t)k * 8 * NN;
      const double* a = b + 4 * NN;
      tb[k].resize(2 * NN);
      ta[k].resize(2 * NN);
      for (int i = 0; i < 2 * NN; ++i) {
        tb[k][i] = b[i] + b[2 * NN + i];
        ta[k][i] = a[i] + a[2 * NN + i];
      }
      Tb[k] = tb[k].data();
      Ta[k] = ta[k].data();
      D[k] = res.data() + 16 + (size_t)R * 8 * NN + (size_t)k * (2 * N);
    }
    lucj_grad_assemble(*G, N, Tb, Ta, D, grad);
  });
}

int ffx_df_chain_energy_grad(ffx_plan plan, const void* vec0, const ffx_df_ham* ham, const ffx_df_ham* obs,
                             double dt, int n_steps, double* energy, double* grad_h, double* grad_J,
                             double* grad_U, void* psi_out, void* workspace, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec0 || !energy || !grad_h || !workspace) throw Error(FFX_EINVAL, "null pointer");
    if (n_steps < 1 || !std::isfinite(dt)) throw Error(FFX_EINVAL, "bad n_steps or dt");
    ffx_plan_s& P = *plan;
    const int N = P.norb, NN = N * N;
    DFHost df = load_df(P, ham);
    DFHost ob = load_df(P, obs);
    const int L = df.L;
    if (L > 0 && (!grad_J || !grad_U)) throw Error(FFX_EINVAL, "null gradient pointer");
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    // result block: per term the transition matrices and the J gradient, then the observable's
    P.results_for(std::max<size_t>(16, (size_t)L * 9 * NN + 4 * NN), s);
    const size_t S = P.state_bytes();
    const size_t Sa = (S + 255) / 256 * 256;
    char* ws = (char*)workspace;
    void* lam = ws;
    void* tmp = ws + Sa;
    void* psiT = ws + 2 * Sa;
    void* lamT = ws + 3 * Sa;
    void* psi = ws + 4 * Sa;  // the reverse sweep uncomputes it; psi_out gets a copy
    double* part = (double*)(ws + 5 * Sa);

    DecompPool pool;
    std::map<std::pair<int, int>, const Decomposition*> cache;
    // script-U(W_to^dag W_from), frames: -1 = lab, 0 = eigenbasis of h, t = U_t
    auto rot = [&](int from, int to) -> const Decomposition* {
      auto key = std::make_pair(from, to);
      auto it = cache.find(key);
      if (it != cache.end()) return it->second;
      std::vector<cd> M;
      if (from < 0)
        M = dagger(N, df.Wm(to));
      else if (to < 0)
        M = df.Wm(from);
      else
        M = matmul(N, dagger(N, df.Wm(to)), df.Wm(from));
      const Decomposition* d = pool.add(N, M);
      cache.emplace(key, d);
      return d;
    };
    // forward: n_steps of S_0 (one-body term first), neighbours merged, the
    // one-body factor carried as the rotation Q(dt) = exp(-i dt h)
    Program fwd;
    {
      std::vector<std::pair<int, double>> m;
      for (int r = 0; r < n_steps; ++r)
        for (int t = 0; t <= L; ++t) {
          if (!m.empty() && m.back().first == t)
            m.back().second += dt;
          else
            m.push_back({t, dt});
        }
      fwd = product_formula_program(df, N, m, pool);
    }
    // costate terms of the observable
    std::vector<Program> terms(ob.L + 1);
    for (int t = 0; t <= ob.L; ++t) {
      const Decomposition* to = pool.add(N, dagger(N, ob.Wm(t)));
      const Decomposition* from = pool.add(N, ob.Wm(t));
      terms[t].rot(to, to);
      terms[t].scale(terms[t].add_diag(df_weight_spec(ob, t)));
      terms[t].rot(from, from);
    }
    // reverse sweep of one step: into frame L, then per term t: undo D_t,
    // move to frame t-1; finally undo the one-body factor Q(dt) on the way
    // back to the lab frame (one rotation, script-U(Q^dag U_1))
    Program first, tail;
    std::vector<Program> undoD(L + 1), link(L + 1);
    if (L >= 1) {
      const Decomposition* d = rot(-1, L);
      first.rot(d, d);
    }
    for (int t = L; t >= 1; --t) {
      undoD[t].phase(undoD[t].add_diag(df_weight_spec(df, t)), +dt);
      if (t >= 2) {
        const Decomposition* d = rot(t, t - 1);
        link[t].rot(d, d);
      }
    }
    {
      std::vector<cd> M = dagger(N, one_body_rotation(df, N, dt));
      if (L >= 1) M = matmul(N, M, df.Wm(1));
      const Decomposition* d = pool.add(N, M);
      tail.rot(d, d);
    }
    HamAction onebody;  // the observable's one-body term, directly when its tables are short
    prepare_one_body(P, obs->h, onebody);
    Upload up(&P, s);
    Compiled c_fwd = compile_program(P, up, fwd, FINAL_STORE, s);
    std::vector<Compiled> c_terms;
    for (int t = 0; t <= ob.L; ++t)
      c_terms.push_back(compile_program(P, up, terms[t], t == 0 ? FINAL_STORE : FINAL_ACCUM, s));
    Compiled c_first = compile_program(P, up, first, FINAL_STORE, s);
    Compiled c_tail = compile_program(P, up, tail, FINAL_STORE, s);
    std::vector<Compiled> c_undoD(L + 1), c_link(L + 1);
    for (int t = L; t >= 1; --t) {
      c_undoD[t] = compile_program(P, up, undoD[t], FINAL_STORE, s);
      if (t >= 2) c_link[t] = compile_program(P, up, link[t], FINAL_STORE, s);
    }
    up.commit();

    // forward and costate
    execute_program(P, c_fwd, vec0, psi, nullptr, s);
    if (psi_out) HIPCHK(hipMemcpyAsync(psi_out, psi, S, hipMemcpyDeviceToDevice, s));
    for (int t = 0; t <= ob.L; ++t) {
      if (t == 0 && onebody.direct)
        apply_one_body_direct(P, onebody, psi, lam, tmp, s);
      else if (t == 0)
        execute_program(P, c_terms[t], psi, lam, nullptr, s);
      else
        execute_program(P, c_terms[t], psi, tmp, lam, s);
    }
    dev::inner(P.c64, psi, lam, P.elems(), P.partials, P.results, s);
    check_launch();
    double e2[2];
    HIPCHK(hipMemcpyAsync(e2, P.results, sizeof(e2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *energy = e2[0];

    auto both = [&](const Compiled& c) {
      execute_program(P, c, psi, psi, nullptr, s);
      execute_program(P, c, lam, lam, nullptr, s);
    };
    auto rdm = [&](double* Tout) { transition_rdm(P, lam, psi, lamT, psiT, part, Tout, s); };
    // device results per step: [t = 1..L: Tb (4N^2), Ta (4N^2), Jg (N^2)] [T_O (4N^2)]
    auto Tb_at = [&](int t) { return P.results + (size_t)(t - 1) * 9 * NN; };
    double* TO = P.results + (size_t)L * 9 * NN;
    std::vector<std::vector<cd>> G(L + 1, std::vector<cd>((size_t)NN, 0.0));
    std::vector<std::vector<double>> Jg(L + 1, std::vector<double>((size_t)NN, 0.0));
    std::vector<cd> GO((size_t)NN, 0.0);
    std::vector<double> res((size_t)L * 9 * NN + 4 * NN);
    for (int step = n_steps - 1; step >= 0; --step) {
      if (L >= 1) both(c_first);
      for (int t = L; t >= 1; --t) {
        double* Tb = Tb_at(t);
        rdm(Tb);
        dev::dc_grad_rows(P.c64, lam, psi, P.dim[0], P.dim[1], P.d_masks[0], P.d_masks[1], N, part, s);
        dev::sum_columns(part, (int)P.dim[0], NN, Tb + 8 * NN, s);
        check_launch();
        both(c_undoD[t]);
        rdm(Tb + 4 * NN);
        if (t >= 2) both(c_link[t]);
      }
      both(c_tail);
      rdm(TO);
      HIPCHK(hipMemcpyAsync(res.data(), P.results, res.size() * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int t = 1; t <= L; ++t) {
        const double* b = res.data() + (size_t)(t - 1) * 9 * NN;
        const double* a = b + 4 * NN;
        const double* j = b + 8 * NN;
        for (int i = 0; i < NN; ++i) {
          G[t][i] += cd(b[2 * i] + b[2 * NN + 2 * i] - a[2 * i] - a[2 * NN + 2 * i],
                        b[2 * i + 1] + b[2 * NN + 2 * i + 1] - a[2 * i + 1] - a[2 * NN + 2 * i + 1]);
          Jg[t][i] += dt * j[i];
        }
      }
      const double* o = res.data() + (size_t)L * 9 * NN;
      for (int i = 0; i < NN; ++i) GO[i] += cd(o[2 * i] + o[2 * NN + 2 * i], o[2 * i + 1] + o[2 * NN + 2 * i + 1]);
    }
    // chain rules; symmetric parameters report the derivative for moving the pair (p, q) and (q, p)
    std::vector<double> gre((size_t)NN), gim((size_t)NN);
    {
      std::vector<cd> K((size_t)NN);
      for (int i = 0; i < NN; ++i) K[i] = cd(0.0, -dt * ham->h[i]);
      expm_param_grad(N, K, GO, gre.data(), gim.data());
      for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q)
          grad_h[p * N + q] = p == q ? -0.5 * dt * gim[p * N + p] : -0.5 * dt * (gim[p * N + q] + gim[q * N + p]);
    }
    std::vector<cd> K0((size_t)NN, 0.0);
    for (int t = 1; t <= L; ++t) {
      double* gu = grad_U + (size_t)(t - 1) * 2 * NN;
      expm_param_grad(N, K0, G[t], gu, gu + NN);
      double* gj = grad_J + (size_t)(t - 1) * NN;
      for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q)
          gj[p * N + q] = p == q ? Jg[t][p * N + p] : Jg[t][p * N + q] + Jg[t][q * N + p];
    }
  });
}

int ffx_timing_enable(ffx_plan plan, int enable) {
  return guard([&] {
    validate_plan(plan);
    DeviceGuard dg(plan->device);
    for (auto& t : plan->timed) {
      HIPCHK(hipEventSynchronize(t.b));
    }
    plan->recycle_timed();
    plan->timing = enable != 0;
  });
}

int ffx_timing_read(ffx_plan plan, int which, double* total_ms, int64_t* launches, double* alg_bytes,
                    double* valu_slots) {
  return guard([&] {
    validate_plan(plan);
    if (which < 0 || which > 5) throw Error(FFX_EINVAL, "bad selector");
    DeviceGuard dg(plan->device);
    double ms = 0, bytes = 0, slots = 0;
    int64_t n = 0;
    for (auto& t : plan->timed) {
      if (t.kind * 2 + t.spin != which) continue;
      HIPCHK(hipEventSynchronize(t.b));
      float e = 0;
      HIPCHK(hipEventElapsedTime(&e, t.a, t.b));
      ms += e;
      bytes += t.alg_bytes;
      slots += t.valu_slots;
      ++n;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    if (alg_bytes) *alg_bytes = bytes;
    if (valu_slots) *valu_slots = slots;
  });
}

}  // extern "C"
