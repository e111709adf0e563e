// CPU checks of libffx's host layer (configuration tables, window and segment
// class tables, packed segments, crossing ranges, Givens decompositions, the
// one-body excitation tables and the small dense helpers), built with g++
// under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_tables.py.  Every table is checked by walking every entry
// against facts derived here independently: bit patterns, fermionic signs from
// the creation-operator ordering, determinants by elimination, reconstruction
// of the unitary from its rotations.  Prints "host checks passed" and exits 0,
// or prints the first failure and exits 1.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "ffx.h"
#include "host.h"

using ffx::cd;

static int g_checks = 0;

#define CHECK(cond, ...)                                   \
  do {                                                     \
    ++g_checks;                                            \
    if (!(cond)) {                                         \
      std::fprintf(stderr, "FAILED %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                   \
      std::fprintf(stderr, "\n");                          \
      std::exit(1);                                        \
    }                                                      \
  } while (0)

static int popc(uint64_t x) { return __builtin_popcountll(x); }

// k-th w-bit pattern with m bits set, ascending integer order
static std::vector<std::vector<int>> patterns(int w) {
  std::vector<std::vector<int>> p(w + 1);
  for (int x = 0; x < (1 << w); ++x) p[popc((uint64_t)x)].push_back(x);
  return p;
}

static void check_strings() {
  for (int N = 1; N <= 32; ++N)
    for (int n = 0; n <= N; ++n) {
      if (ffx::binom(N, n) > 200000) continue;
      const auto s = ffx::make_strings(N, n);
      CHECK((int64_t)s.size() == ffx::binom(N, n), "count N=%d n=%d", N, n);
      for (size_t i = 0; i < s.size(); ++i) {
        CHECK(popc(s[i]) == n && (N == 64 || s[i] < (1ull << N)), "string N=%d n=%d i=%zu", N, n, i);
        if (i) CHECK(s[i] > s[i - 1], "order N=%d n=%d i=%zu", N, n, i);
      }
    }
}

// random unitary: Gram-Schmidt on a complex Gaussian matrix (columns)
static std::vector<cd> random_unitary(int N, std::mt19937_64& rng, bool real) {
  std::normal_distribution<double> g;
  std::vector<cd> U((size_t)N * N);
  for (auto& x : U) x = real ? cd(g(rng), 0.0) : cd(g(rng), g(rng));
  for (int j = 0; j < N; ++j) {
    for (int k = 0; k < j; ++k) {
      cd dot = 0;
      for (int i = 0; i < N; ++i) dot += std::conj(U[i * N + k]) * U[i * N + j];
      for (int i = 0; i < N; ++i) U[i * N + j] -= dot * U[i * N + k];
    }
    double nr = 0;
    for (int i = 0; i < N; ++i) nr += std::norm(U[i * N + j]);
    nr = std::sqrt(nr);
    for (int i = 0; i < N; ++i) U[i * N + j] /= nr;
  }
  return U;
}

static void check_givens() {
  std::mt19937_64 rng(7);
  for (int N : {1, 2, 3, 5, 8, 13, 16, 19, 24, 32})
    for (bool real : {false, true}) {
      const auto U = random_unitary(N, rng, real);
      CHECK(ffx::unitarity_defect(N, U.data()) < 1e-13, "unitary N=%d", N);
      const ffx::Decomposition d = ffx::givens_decompose(N, U.data());
      CHECK((int)d.rots.size() <= N * (N - 1) / 2 && (int)d.phase.size() == N, "sizes N=%d", N);
      // rebuild: M = diag(exp(i phase)) G_K ... G_1, G_k acting on (p, p+1) as [[c, s], [-conj(s), c]]
      std::vector<cd> M((size_t)N * N, 0.0);
      for (int i = 0; i < N; ++i) M[i * N + i] = 1.0;
      for (const auto& r : d.rots) {
        CHECK(r.p >= 0 && r.p + 1 < N, "position N=%d", N);
        CHECK(std::abs(r.c * r.c + std::norm(r.s) - 1.0) < 1e-13, "2x2 block not unitary N=%d", N);
        for (int j = 0; j < N; ++j) {
          const cd x = M[r.p * N + j], y = M[(r.p + 1) * N + j];
          M[r.p * N + j] = r.c * x + r.s * y;
          M[(r.p + 1) * N + j] = -std::conj(r.s) * x + r.c * y;
        }
      }
      double err = 0;
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) err = std::max(err, std::abs(std::exp(cd(0, d.phase[i])) * M[i * N + j] - U[i * N + j]));
      CHECK(err < 1e-12, "reconstruction N=%d real=%d err=%g", N, (int)real, err);
      if (real) CHECK(d.real, "real flag N=%d", N);
    }
  bool threw = false;
  std::vector<cd> bad(9, 1.0);
  try {
    ffx::givens_decompose(3, bad.data());
  } catch (const ffx::Error& e) {
    threw = e.code == FFX_ENOTUNITARY;
  }
  CHECK(threw, "non-unitary input accepted");
}

// Schedules of a decomposition whose rotations cross a segment window [0, wt):
// every rotation exactly once, after the rotations it depends on (those
// sharing an orbital and earlier in the list), stages inside [a, a + w) within
// the segment window, window passes inside [a, a + W) taking a crossing
// rotation; and the beam search needs no more stages than the greedy order
// (stages first, then one whole-spin window pass when none can progress).
static void check_cross_schedules() {
  std::mt19937_64 rng(11);
  for (int N : {8, 11, 17, 18}) {
    const auto U = random_unitary(N, rng, true);
    const ffx::Decomposition d = ffx::givens_decompose(N, U.data());
    const int n = (int)d.rots.size();
    for (int wt : {N - 1, N - 2, N - 3, 6}) {
      const int w = std::min(6, wt);
      const auto sp = ffx::schedule_windows_cross(d.rots, N, wt, w, 6, 300, 3);
      CHECK(!sp.empty(), "cross schedule found N=%d wt=%d", N, wt);
      std::vector<int> when(n, -1);
      int step = 0, stages = 0;
      for (const auto& p : sp) {
        const int lo = p.a, hi = p.a + (p.win ? 6 : w);
        CHECK(lo >= 0 && hi <= (p.win ? N : wt), "window bounds N=%d wt=%d", N, wt);
        bool crosses = false;
        for (int i : p.idx) {
          CHECK(i >= 0 && i < n && when[i] < 0, "rotation once N=%d wt=%d", N, wt);
          CHECK(d.rots[i].p >= lo && d.rots[i].p + 1 < hi, "rotation inside its window N=%d wt=%d", N, wt);
          crosses = crosses || d.rots[i].p + 1 >= wt;
          when[i] = step++;
        }
        if (p.win) CHECK(crosses, "window pass without a crossing rotation N=%d wt=%d", N, wt);
        else ++stages;
      }
      for (int i = 0; i < n; ++i) {
        CHECK(when[i] >= 0, "rotation scheduled N=%d wt=%d", N, wt);
        for (int j = 0; j < i; ++j) {
          const int pi = d.rots[i].p, pj = d.rots[j].p;
          if (pj == pi || pj == pi + 1 || pj + 1 == pi) CHECK(when[j] < when[i], "dependency order N=%d wt=%d", N, wt);
        }
      }
      // the greedy order, for comparison
      std::vector<char> done(n, 0);
      int greedy = 0, left = n;
      while (left > 0) {
        bool progressed = true;
        while (progressed) {
          progressed = false;
          std::vector<int> best;
          for (int a = 0; a + w <= wt; ++a) {
            std::vector<int> t;
            std::vector<char> taken(n, 0);
            for (int i = 0; i < n; ++i) {
              if (done[i] || d.rots[i].p < a || d.rots[i].p + 1 >= a + w) continue;
              bool ok = true;
              for (int j = 0; j < i; ++j) {
                const int pi = d.rots[i].p, pj = d.rots[j].p;
                if ((pj == pi || pj == pi + 1 || pj + 1 == pi) && !done[j] && !taken[j]) ok = false;
              }
              if (ok) {
                taken[i] = 1;
                t.push_back(i);
              }
            }
            if (t.size() > best.size()) best = t;
          }
          if (!best.empty()) {
            for (int i : best) done[i] = 1;
            left -= (int)best.size();
            ++greedy;
            progressed = true;
          }
        }
        if (left == 0) break;
        std::vector<int> best;
        for (int a = 0; a + 6 <= N; ++a) {
          std::vector<int> t;
          std::vector<char> taken(n, 0);
          for (int i = 0; i < n; ++i) {
            if (done[i] || d.rots[i].p < a || d.rots[i].p + 1 >= a + 6) continue;
            bool ok = true;
            for (int j = 0; j < i; ++j) {
              const int pi = d.rots[i].p, pj = d.rots[j].p;
              if ((pj == pi || pj == pi + 1 || pj + 1 == pi) && !done[j] && !taken[j]) ok = false;
            }
            if (ok) {
              taken[i] = 1;
              t.push_back(i);
            }
          }
          if (t.size() > best.size()) best = t;
        }
        for (int i : best) done[i] = 1;
        left -= (int)best.size();
      }
      CHECK(stages <= greedy, "beam stages %d > greedy %d at N=%d wt=%d", stages, greedy, N, wt);
    }
    // the pair straddling the window as a two-orbital window (applied at load): one rotation each time
    const int wt = N - 1;
    const auto sp = ffx::schedule_windows_cross(d.rots, N, wt, 6, 2, 300, 3);
    CHECK(!sp.empty(), "at-load schedule found N=%d", N);
    std::vector<int> when(n, -1);
    int step = 0;
    for (const auto& p : sp) {
      if (p.win) CHECK(p.idx.size() == 1 && d.rots[p.idx[0]].p == wt - 1, "at-load step N=%d", N);
      for (int i : p.idx) {
        CHECK(when[i] < 0, "at-load rotation once N=%d", N);
        when[i] = step++;
      }
    }
    for (int i = 0; i < n; ++i) {
      CHECK(when[i] >= 0, "at-load rotation scheduled N=%d", N);
      for (int j = 0; j < i; ++j) {
        const int pi = d.rots[i].p, pj = d.rots[j].p;
        if (pj == pi || pj == pi + 1 || pj + 1 == pi) CHECK(when[j] < when[i], "at-load order N=%d", N);
      }
    }
  }
}

static void check_window_tables() {
  for (auto [N, n] : std::vector<std::pair<int, int>>{{6, 3}, {8, 4}, {9, 2}, {10, 5}, {12, 6}, {13, 4}, {16, 8},
                                                       {16, 1}, {7, 0}, {7, 7}}) {
    const auto strs = ffx::make_strings(N, n);
    std::map<uint64_t, int> addr;
    for (size_t i = 0; i < strs.size(); ++i) addr[strs[i]] = (int)i;
    const int w = std::min(N, 6);
    const auto pats = patterns(w);
    for (int a = 0; a + w <= N; ++a) {
      const ffx::WindowTable t = ffx::build_window_table(strs, N, n, a, w);
      const uint64_t wm = ((1ull << w) - 1) << a;
      std::vector<int> seen(strs.size(), 0);
      for (size_t c = 0; c < t.chunk_m.size(); ++c) {
        const int m = t.chunk_m[c], off = t.chunk_off[c], live = t.chunk_n[c];
        CHECK(live >= 1 && live <= 64, "live lanes N=%d a=%d", N, a);
        for (int lane = 0; lane < 64; ++lane) {
          uint64_t outside = 0;
          for (int k = 0; k < (int)pats[m].size(); ++k) {
            const int ad = t.tab[off + k * 64 + lane];
            if (lane >= live) {
              CHECK(ad == -1, "padding lane N=%d a=%d", N, a);
              continue;
            }
            CHECK(ad >= 0 && ad < (int)strs.size(), "address N=%d a=%d", N, a);
            const uint64_t x = strs[ad];
            CHECK((int)((x & wm) >> a) == pats[m][k], "member pattern N=%d a=%d m=%d k=%d", N, a, m, k);
            if (k == 0) outside = x & ~wm;
            CHECK((x & ~wm) == outside, "class outside bits N=%d a=%d", N, a);
            ++seen[ad];
          }
        }
      }
      for (size_t i = 0; i < strs.size(); ++i) CHECK(seen[i] == 1, "coverage N=%d n=%d a=%d i=%zu", N, n, a, i);
      CHECK(t.cls.size() > 0, "no classes");
    }
  }
}

// every class member of every register window of a segment: positions inside
// the segment, in-window patterns in order, shared bits outside the window,
// and every configuration with 0 < m < w reached exactly once
static void check_segment(const std::vector<uint64_t>& seg, int wt, int w, int group, const char* what) {
  const auto pats = patterns(w);
  for (int a = 0; a + w <= wt; ++a) {
    ffx::SegWindowTable t = ffx::build_seg_window(seg, wt, a, w, group);
    const uint64_t wm = ((1ull << w) - 1) << a;
    auto walk = [&](const ffx::SegWindowTable& tb, std::vector<int>& seen, std::multiset<int>& codes) {
      CHECK(tb.code.size() == 64 * tb.chunk_m.size(), "%s: table shape", what);
      for (size_t c = 0; c < tb.chunk_m.size(); ++c)
        for (int lane = 0; lane < 64; ++lane) {
          const int code = tb.code[c * 64 + lane];
          if (code < 0) continue;
          codes.insert(code * 16 + tb.chunk_m[c]);
          const int m = tb.chunk_m[c], cbase = code >> 5, l = code & 31;
          CHECK(m > 0 && m < w && l < tb.nl1, "%s: class m=%d l=%d", what, m, l);
          uint64_t outside = 0;
          for (int k = 0; k < (int)pats[m].size(); ++k) {
            const int pos = cbase + tb.mt[tb.mt[m * tb.nl1 + l] + k];
            CHECK(pos >= 0 && pos < (int)seg.size(), "%s: position a=%d", what, a);
            const uint64_t x = seg[pos];
            CHECK((int)((x & wm) >> a) == pats[m][k], "%s: pattern a=%d m=%d k=%d", what, a, m, k);
            CHECK(popc(x & ((1ull << a) - 1)) == l, "%s: electrons below the window", what);
            if (k == 0) outside = x & ~wm;
            CHECK((x & ~wm) == outside, "%s: class outside bits a=%d", what, a);
            ++seen[pos];
          }
        }
    };
    std::vector<int> seen(seg.size(), 0);
    std::multiset<int> codes;
    walk(t, seen, codes);
    for (size_t i = 0; i < seg.size(); ++i) {
      const int m = popc(seg[i] & wm);
      CHECK(seen[i] == ((m > 0 && m < w) ? 1 : 0), "%s: coverage a=%d i=%zu m=%d", what, a, i, m);
    }
    // the SIMD balancing only reorders chunks
    for (int nwaves : {12, 16}) {
      ffx::SegWindowTable b = t;
      ffx::balance_seg_window(b, w, nwaves);
      std::vector<int> seen2(seg.size(), 0);
      std::multiset<int> codes2;
      walk(b, seen2, codes2);
      CHECK(codes2 == codes && seen2 == seen, "%s: balancing changed the classes", what);
    }
    // packed codes: the base and the absolute index of the class's offset
    // table, with the window's tables placed at an arbitrary start in the block
    {
      const int mt_off = 4 * (a + 1);
      const std::vector<int> packed = ffx::pack_class_codes(t, mt_off);
      CHECK(packed.size() == t.code.size(), "%s: packed code count", what);
      for (size_t c = 0; c < t.chunk_m.size(); ++c)
        for (int lane = 0; lane < 64; ++lane) {
          const int code = t.code[c * 64 + lane], pk = packed[c * 64 + lane];
          if (code < 0) {
            CHECK(pk == -1, "%s: packed padding", what);
            continue;
          }
          const int m = t.chunk_m[c];
          CHECK((pk >> ffx::kCodeMoffBits) == (code >> 5), "%s: packed base a=%d", what, a);
          CHECK((pk & ((1 << ffx::kCodeMoffBits) - 1)) == mt_off + t.mt[m * t.nl1 + (code & 31)],
                "%s: packed table index a=%d", what, a);
        }
    }
    // replication over rows shifts the bases by whole rows
    const int R = 3;
    ffx::SegWindowTable rep = ffx::replicate_seg_window(t, w, R, (int)seg.size());
    std::vector<uint64_t> rows;
    for (int r = 0; r < R; ++r) rows.insert(rows.end(), seg.begin(), seg.end());
    size_t n_rep = 0;
    for (size_t c = 0; c < rep.chunk_m.size(); ++c)
      for (int lane = 0; lane < 64; ++lane)
        if (rep.code[c * 64 + lane] >= 0) ++n_rep;
    CHECK(n_rep == R * codes.size(), "%s: replicated class count", what);
  }
}

static void check_segments() {
  struct Case {
    int N, n;
  };
  for (Case cs : std::vector<Case>{{8, 4}, {10, 3}, {12, 6}, {14, 7}, {16, 8}, {18, 9}, {20, 3}, {24, 2}, {28, 4},
                                   {32, 4}, {32, 2}, {9, 0}, {9, 9}}) {
    const auto strs = ffx::make_strings(cs.N, cs.n);
    const int w = 6;
    for (int wt = std::max(0, cs.N - 4); wt <= cs.N; ++wt) {
      const auto runs = ffx::segment_runs(strs, wt);
      // runs: contiguous, cover everything, share the bits >= wt
      int next = 0;
      for (const auto& r : runs) {
        CHECK(r.first == next && r.second >= 1, "runs contiguous N=%d wt=%d", cs.N, wt);
        for (int i = r.first; i < r.first + r.second; ++i)
          CHECK((strs[i] >> wt) == (strs[r.first] >> wt), "run high bits N=%d wt=%d", cs.N, wt);
        if (r.first > 0) CHECK((strs[r.first] >> wt) != (strs[r.first - 1] >> wt), "run maximal N=%d wt=%d", cs.N, wt);
        next = r.first + r.second;
      }
      CHECK(next == (int)strs.size(), "runs cover N=%d wt=%d", cs.N, wt);
      const int ww = std::min(w, wt);
      char what[96];
      if (ww >= 2) {
        for (size_t g = 0; g < runs.size(); g += std::max<size_t>(1, runs.size() / 7)) {
          std::vector<uint64_t> sub(strs.begin() + runs[g].first, strs.begin() + runs[g].first + runs[g].second);
          std::snprintf(what, sizeof what, "run N=%d n=%d wt=%d g=%zu", cs.N, cs.n, wt, g);
          check_segment(sub, wt, ww, 8, what);
        }
        // packed segments: consecutive runs back to back up to a cap
        for (int64_t cap : {(int64_t)64, (int64_t)1000, (int64_t)6435}) {
          const auto groups = ffx::pack_runs(runs, cap);
          int nx = 0;
          for (const auto& gr : groups) {
            CHECK(gr.first == nx, "packed contiguous");
            nx += gr.second;
          }
          CHECK(nx == (int)strs.size(), "packed cover");
          for (size_t g = 0; g < groups.size(); g += std::max<size_t>(1, groups.size() / 5)) {
            std::vector<uint64_t> sub(strs.begin() + groups[g].first,
                                      strs.begin() + groups[g].first + groups[g].second);
            std::snprintf(what, sizeof what, "packed N=%d n=%d wt=%d cap=%lld g=%zu", cs.N, cs.n, wt, (long long)cap, g);
            check_segment(sub, wt, ww, 16, what);
          }
        }
      }
      // crossing ranges of the rotation on (wt - 1, wt): own and partner ranges pair every configuration
      // holding exactly one of the two orbitals with its image under the exchange, each exactly once
      if (wt >= 1 && wt < cs.N && runs.size() > 1) {
        const auto cr = ffx::crossing_ranges(strs, runs, wt, cs.n);
        const uint64_t bl = 1ull << (wt - 1), bh = 1ull << wt;
        std::vector<int> own(strs.size(), 0);
        for (size_t g = 0; g < runs.size(); ++g) {
          if (!cr[g].has) continue;
          for (int i = 0; i < cr[g].cnt; ++i) {
            const uint64_t x = strs[runs[g].first + cr[g].lo + i], y = strs[cr[g].peer + i];
            if (cr[g].role == 0)
              CHECK((x & bl) && !(x & bh) && (y & bh) && !(y & bl), "crossing roles N=%d wt=%d", cs.N, wt);
            else
              CHECK((x & bh) && !(x & bl) && (y & bl) && !(y & bh), "crossing roles N=%d wt=%d", cs.N, wt);
            CHECK((x ^ bl ^ bh) == y, "crossing partner N=%d wt=%d g=%zu i=%d", cs.N, wt, g, i);
            ++own[runs[g].first + cr[g].lo + i];
          }
        }
        for (size_t i = 0; i < strs.size(); ++i) {
          const bool one = ((strs[i] & bl) != 0) != ((strs[i] & bh) != 0);
          CHECK(own[i] == (one ? 1 : 0), "crossing coverage N=%d wt=%d i=%zu", cs.N, wt, i);
        }
      }
    }
  }
}

// a^dag_p a_q |I> by the creation-operator ordering: annihilating q passes the
// occupied orbitals below q, creating p passes those below p in I - q
static void check_one_body_tables() {
  std::mt19937_64 rng(11);
  std::normal_distribution<double> g;
  for (auto [N, n] : std::vector<std::pair<int, int>>{{5, 2}, {6, 3}, {8, 4}, {9, 1}, {7, 0}, {7, 7}, {10, 3}}) {
    std::vector<double> h((size_t)N * N, 0.0);
    for (int p = 0; p < N; ++p)
      for (int q = p; q < N; ++q) {
        const double v = (q == p + 3) ? 0.0 : g(rng);  // some zero couplings
        h[p * N + q] = h[q * N + p] = v;
      }
    const auto strs = ffx::make_strings(N, n);
    const int d = (int)strs.size();
    std::map<uint64_t, int> addr;
    for (int i = 0; i < d; ++i) addr[strs[i]] = i;
    std::vector<double> ref((size_t)d * d, 0.0);  // ref[J][I]
    for (int I = 0; I < d; ++I)
      for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q) {
          const uint64_t x = strs[I];
          if (!((x >> q) & 1)) continue;
          const uint64_t y = x & ~(1ull << q);
          if ((y >> p) & 1) continue;
          const int s1 = popc(x & ((1ull << q) - 1)), s2 = popc(y & ((1ull << p) - 1));
          const uint64_t z = y | (1ull << p);
          ref[(size_t)addr[z] * d + I] += ((s1 + s2) & 1 ? -1.0 : 1.0) * h[p * N + q];
        }
    const ffx::OneBodyTable t = ffx::build_one_body_table(N, strs, h);
    CHECK((int)t.off.size() == d + 1 && t.off[0] == 0, "one-body table shape N=%d", N);
    std::vector<double> got((size_t)d * d, 0.0);
    for (int J = 0; J < d; ++J)
      for (int64_t e = t.off[J]; e < t.off[J + 1]; ++e) {
        CHECK(t.src[e] >= 0 && t.src[e] < d, "one-body source N=%d", N);
        got[(size_t)J * d + t.src[e]] += t.coef[e];
      }
    double err = 0;
    for (size_t i = 0; i < got.size(); ++i) err = std::max(err, std::abs(got[i] - ref[i]));
    CHECK(err < 1e-13, "one-body table N=%d n=%d err=%g", N, n, err);
  }
}

static cd det_elim(std::vector<cd> A, int n) {
  cd det = 1.0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int p = k + 1; p < n; ++p)
      if (std::abs(A[p * n + k]) > std::abs(A[piv * n + k])) piv = p;
    if (piv != k) {
      for (int q = 0; q < n; ++q) std::swap(A[k * n + q], A[piv * n + q]);
      det = -det;
    }
    det *= A[k * n + k];
    if (A[k * n + k] == 0.0) return 0.0;
    for (int p = k + 1; p < n; ++p) {
      const cd f = A[p * n + k] / A[k * n + k];
      for (int q = k; q < n; ++q) A[p * n + q] -= f * A[k * n + q];
    }
  }
  return det;
}

static void check_dense_helpers() {
  std::mt19937_64 rng(5);
  std::normal_distribution<double> g;
  for (int N : {1, 3, 8, 16}) {
    // Hermitian eigendecomposition reconstructs A
    std::vector<cd> A((size_t)N * N);
    for (int i = 0; i < N; ++i)
      for (int j = i; j < N; ++j) {
        const cd v = i == j ? cd(g(rng), 0) : cd(g(rng), g(rng));
        A[i * N + j] = v;
        A[j * N + i] = std::conj(v);
      }
    std::vector<double> w;
    std::vector<cd> W;
    ffx::eigh(N, A, w, W);
    double err = 0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        cd s = 0;
        for (int k = 0; k < N; ++k) s += W[i * N + k] * w[k] * std::conj(W[j * N + k]);
        err = std::max(err, std::abs(s - A[i * N + j]));
      }
    CHECK(err < 1e-11, "eigh N=%d err=%g", N, err);
    // expm of an anti-Hermitian K against its Taylor series at small norm
    std::vector<cd> K((size_t)N * N);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) K[i * N + j] = 0.05 * (A[i * N + j] * cd(0, 1));
    const auto E = ffx::expm_antihermitian(N, K);
    std::vector<cd> T((size_t)N * N, 0.0), P((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i) T[i * N + i] = P[i * N + i] = 1.0;
    for (int k = 1; k < 30; ++k) {
      P = ffx::matmul(N, P, K);
      for (auto& x : P) x /= (double)k;
      for (size_t i = 0; i < T.size(); ++i) T[i] += P[i];
    }
    err = 0;
    for (size_t i = 0; i < T.size(); ++i) err = std::max(err, std::abs(T[i] - E[i]));
    CHECK(err < 1e-12, "expm N=%d err=%g", N, err);
  }
  // Slater column minors against determinants by elimination
  for (auto [N, n] : std::vector<std::pair<int, int>>{{6, 3}, {8, 2}, {9, 5}, {5, 0}}) {
    const auto U = random_unitary(N, rng, false);
    const auto strs = ffx::make_strings(N, n);
    const auto v = ffx::slater_column_minors(N, n, U, strs);
    for (size_t J = 0; J < strs.size(); ++J) {
      std::vector<cd> M((size_t)n * n);
      int r = 0;
      for (int p = 0; p < N; ++p)
        if ((strs[J] >> p) & 1) {
          for (int c = 0; c < n; ++c) M[r * n + c] = U[p * N + c];
          ++r;
        }
      CHECK(std::abs(v[J] - det_elim(M, n)) < 1e-12, "slater minor N=%d n=%d J=%zu", N, n, J);
    }
  }
  // Bessel functions of the first kind at tabulated points
  const auto j1 = ffx::bessel_j_series(1.0, 3);
  CHECK(std::abs(j1[0] - 0.7651976865579666) < 1e-14 && std::abs(j1[1] - 0.4400505857449335) < 1e-14,
        "Bessel J_k(1)");
  const auto j10 = ffx::bessel_j_series(10.0, 6);
  CHECK(std::abs(j10[0] + 0.2459357644513483) < 1e-13 && std::abs(j10[5] + 0.2340615281867936) < 1e-13,
        "Bessel J_k(10)");
}

int main() {
  check_strings();
  check_givens();
  check_cross_schedules();
  check_window_tables();
  check_segments();
  check_one_body_tables();
  check_dense_helpers();
  std::printf("host checks passed (%d)\n", g_checks);
  return 0;
}
