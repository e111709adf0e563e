// Host-side building blocks of libffx (see host.h).
#include "host.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <unordered_map>

#include "ffx.h"

namespace ffx {

int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 0; i < k; ++i) r = r * (n - i) / (i + 1);
  return r;
}

std::vector<uint64_t> make_strings(int norb, int n) {
  std::vector<uint64_t> out;
  out.reserve((size_t)binom(norb, n));
  if (n == 0) {
    out.push_back(0);
    return out;
  }
  uint64_t x = (n == 64) ? ~0ull : ((1ull << n) - 1);
  const uint64_t limit = 1ull << norb;
  while (x < limit) {
    out.push_back(x);
    // Gosper's hack: next larger integer with the same popcount
    uint64_t u = x & (~x + 1);
    uint64_t v = x + u;
    if (v == 0) break;
    x = v + (((v ^ x) / u) >> 2);
  }
  return out;
}

double unitarity_defect(int norb, const cd* U) {
  double worst = 0;
  for (int i = 0; i < norb; ++i)
    for (int j = 0; j < norb; ++j) {
      cd acc = 0;
      for (int k = 0; k < norb; ++k) acc += std::conj(U[k * norb + i]) * U[k * norb + j];
      worst = std::max(worst, std::abs(acc - (i == j ? 1.0 : 0.0)));
    }
  return worst;
}

// Column elimination by right multiplication: for rows i = N-1 .. 1, zero
// V[i][j] for j = 0 .. i-1 with a rotation R of columns (j, j+1).  Then
// U R_1 ... R_K = D, i.e. U = D R_K^dag ... R_1^dag, and the state sees
// G_k = R_k^dag in the recorded order.
Decomposition givens_decompose(int norb, const cd* U) {
  if (unitarity_defect(norb, U) > 1e-10) throw Error(FFX_ENOTUNITARY, "orbital rotation is not unitary");
  std::vector<cd> V(U, U + norb * norb);
  Decomposition d;
  bool real = true;
  for (int k = 0; k < norb * norb; ++k)
    if (U[k].imag() != 0.0) real = false;
  for (int i = norb - 1; i >= 1; --i) {
    for (int j = 0; j < i; ++j) {
      cd a = V[i * norb + j], b = V[i * norb + j + 1];
      double aa = std::abs(a), ab = std::abs(b);
      double r = std::hypot(aa, ab);
      double c;
      cd s;
      if (r == 0.0) {
        c = 1.0;
        s = 0.0;
      } else if (ab == 0.0) {
        c = 0.0;
        s = 1.0;
      } else {
        c = ab / r;
        s = std::conj(a) * (b / ab) / r;
      }
      // V <- V R on columns (j, j+1), R = [[c, s], [-conj(s), c]]
      for (int row = 0; row < norb; ++row) {
        cd x = V[row * norb + j], y = V[row * norb + j + 1];
        V[row * norb + j] = c * x - std::conj(s) * y;
        V[row * norb + j + 1] = s * x + c * y;
      }
      V[i * norb + j] = 0.0;
      d.rots.push_back(Givens{j, c, -s});
    }
  }
  d.phase.resize(norb);
  for (int p = 0; p < norb; ++p) d.phase[p] = std::arg(V[p * norb + p]);
  if (real) {
    for (auto& g : d.rots) g.s = cd(g.s.real(), 0.0);
    for (int p = 0; p < norb; ++p) d.phase[p] = (V[p * norb + p].real() < 0) ? M_PI : 0.0;
  }
  d.real = real;
  return d;
}

std::vector<Pass> schedule_windows(const std::vector<Givens>& rots, int norb, int w) {
  const int n = (int)rots.size();
  std::vector<std::vector<int>> deps(n);
  std::vector<int> last(norb, -1);
  for (int i = 0; i < n; ++i) {
    int p = rots[i].p;
    for (int q : {p, p + 1})
      if (last[q] >= 0) deps[i].push_back(last[q]);
    last[p] = last[p + 1] = i;
  }
  std::vector<char> done(n, 0);
  int remaining = n;
  std::vector<Pass> out;
  while (remaining > 0) {
    int best_a = -1;
    std::vector<char> best;
    int best_count = -1;
    for (int a = 0; a + w <= norb; ++a) {
      std::vector<char> taken(n, 0);
      int count = 0;
      // one ordered scan suffices: dependencies point backwards
      for (int i = 0; i < n; ++i) {
        if (done[i]) continue;
        int p = rots[i].p;
        if (p < a || p + 1 >= a + w) continue;
        bool ok = true;
        for (int dd : deps[i])
          if (!done[dd] && !taken[dd]) {
            ok = false;
            break;
          }
        if (ok) {
          taken[i] = 1;
          ++count;
        }
      }
      if (count > best_count) {
        best_count = count;
        best_a = a;
        best = taken;
      }
    }
    Pass ps;
    ps.a = best_a;
    for (int i = 0; i < n; ++i)
      if (best[i]) {
        ps.idx.push_back(i);
        done[i] = 1;
      }
    remaining -= best_count;
    out.push_back(std::move(ps));
  }
  return out;
}

std::vector<Pass> schedule_windows_beam(const std::vector<Givens>& rots, int norb, int w, int beam) {
  const int n = (int)rots.size();
  std::vector<std::vector<int>> deps(n);
  std::vector<int> last(norb, -1);
  for (int i = 0; i < n; ++i) {
    const int p = rots[i].p;
    if (p < 0 || p + 1 >= norb) throw Error(FFX_EINVAL, "rotation outside the orbitals");
    for (int q : {p, p + 1})
      if (last[q] >= 0) deps[i].push_back(last[q]);
    last[p] = last[p + 1] = i;
  }
  using Set = std::vector<uint64_t>;
  const int words = (n + 63) / 64;
  auto has = [](const Set& d, int i) { return (d[i >> 6] >> (i & 63)) & 1ull; };
  // the rotations inside [a, a + w) whose predecessors are applied or taken
  auto take = [&](const Set& d, int a) {
    std::vector<int> out;
    std::vector<char> taken(n, 0);
    for (int i = 0; i < n; ++i) {
      if (has(d, i)) continue;
      const int p = rots[i].p;
      if (p < a || p + 1 >= a + w) continue;
      bool ok = true;
      for (int dd : deps[i])
        if (!has(d, dd) && !taken[dd]) {
          ok = false;
          break;
        }
      if (ok) {
        taken[i] = 1;
        out.push_back(i);
      }
    }
    return out;
  };
  struct Node {
    int count;
    std::vector<Pass> hist;
  };
  std::vector<std::pair<Set, Node>> front{{Set(words, 0), Node{0, {}}}};
  if (n == 0) return {};
  for (int step = 0; step < n; ++step) {
    std::map<Set, Node> next;  // ordered: the search is deterministic
    for (const auto& fn : front)
      for (int a = 0; a + w <= norb; ++a) {
        std::vector<int> t = take(fn.first, a);
        if (t.empty()) continue;
        Set d = fn.first;
        for (int i : t) d[i >> 6] |= 1ull << (i & 63);
        if (next.count(d)) continue;
        Node nd{fn.second.count + (int)t.size(), fn.second.hist};
        nd.hist.push_back(Pass{a, std::move(t)});
        next.emplace(std::move(d), std::move(nd));
      }
    std::vector<std::pair<Set, Node>> v(next.begin(), next.end());
    std::stable_sort(v.begin(), v.end(), [](const auto& x, const auto& y) { return x.second.count > y.second.count; });
    if (!v.empty() && v[0].second.count == n) return v[0].second.hist;
    if ((int)v.size() > beam) v.resize(beam);
    if (v.empty()) break;
    front = std::move(v);
  }
  return schedule_windows(rots, norb, w);
}

std::vector<SchedPass> schedule_windows_cross(const std::vector<Givens>& rots, int norb, int wt, int w, int W,
                                              int beam, int win_cost,
                                              const std::function<bool(const std::vector<int>&)>* shaped) {
  const int n = (int)rots.size();
  if (n == 0 || win_cost < 1) return {};
  std::vector<std::vector<int>> deps(n);
  std::vector<int> last(norb, -1);
  for (int i = 0; i < n; ++i) {
    const int p = rots[i].p;
    if (p < 0 || p + 1 >= norb) throw Error(FFX_EINVAL, "rotation outside the orbitals");
    for (int q : {p, p + 1})
      if (last[q] >= 0) deps[i].push_back(last[q]);
    last[p] = last[p + 1] = i;
  }
  using Set = std::vector<uint64_t>;
  const int words = (n + 63) / 64;
  auto has = [](const Set& d, int i) { return (d[i >> 6] >> (i & 63)) & 1ull; };
  // the rotations inside [a, a + width) whose predecessors are applied or taken
  auto take = [&](const Set& d, int a, int width) {
    std::vector<int> out;
    std::vector<char> taken(n, 0);
    for (int i = 0; i < n; ++i) {
      if (has(d, i)) continue;
      const int p = rots[i].p;
      if (p < a || p + 1 >= a + width) continue;
      bool ok = true;
      for (int dd : deps[i])
        if (!has(d, dd) && !taken[dd]) {
          ok = false;
          break;
        }
      if (ok) {
        taken[i] = 1;
        out.push_back(i);
      }
    }
    return out;
  };
  struct Node {
    int count;
    std::vector<SchedPass> hist;
  };
  // states by total cost; a state reached before at a lower or equal cost is not kept again
  std::map<int, std::map<Set, Node>> bucket;
  std::map<Set, int> seen;
  bucket[0].emplace(Set(words, 0), Node{0, {}});
  seen[Set(words, 0)] = 0;
  const int max_cost = 4 * n + 16;
  for (auto it = bucket.begin(); it != bucket.end() && it->first <= max_cost; it = bucket.erase(it)) {
    const int cost = it->first;
    std::vector<std::pair<Set, Node>> v;
    for (auto& sn : it->second)
      if (seen[sn.first] == cost) v.push_back(sn);  // (reached at a lower cost since: stale)
    std::stable_sort(v.begin(), v.end(), [](const auto& x, const auto& y) { return x.second.count > y.second.count; });
    if ((int)v.size() > beam) v.resize(beam);
    for (const auto& sn : v)
      if (sn.second.count == n) return sn.second.hist;
    auto push = [&](const Set& d0, const Node& nd0, bool win, int a, std::vector<int> t, int c) {
      Set d = d0;
      for (int i : t) d[i >> 6] |= 1ull << (i & 63);
      auto sit = seen.find(d);
      if (sit != seen.end() && sit->second <= c) return;
      seen[d] = c;
      Node nd{nd0.count + (int)t.size(), nd0.hist};
      nd.hist.push_back(SchedPass{win, a, std::move(t)});
      bucket[c][d] = std::move(nd);
    };
    for (const auto& sn : v) {
      for (int a = 0; a + w <= wt; ++a) {
        std::vector<int> t = take(sn.first, a, w);
        if (t.empty()) continue;
        int c = 1;
        if (shaped) {
          std::vector<int> pos;
          for (int i : t) pos.push_back(rots[i].p - a);
          if (!(*shaped)(pos)) c = 2;
        }
        push(sn.first, sn.second, false, a, std::move(t), cost + c);
      }
      for (int a = 0; a + W <= norb; ++a) {
        std::vector<int> t = take(sn.first, a, W);
        bool crosses = false;
        for (int i : t) crosses = crosses || rots[i].p + 1 >= wt;
        if (crosses) push(sn.first, sn.second, true, a, std::move(t), cost + win_cost);
      }
    }
  }
  return {};
}

WindowTable build_window_table(const std::vector<uint64_t>& strs, int norb, int n, int a, int w) {
  (void)norb;
  (void)n;
  WindowTable t;
  t.a = a;
  t.w = w;
  const uint64_t wmask = ((1ull << w) - 1) << a;
  // in-window pattern -> rank among patterns with the same popcount
  std::vector<int> prank(1 << w, -1);
  {
    std::vector<int> cnt(w + 1, 0);
    for (int x = 0; x < (1 << w); ++x) prank[x] = cnt[__builtin_popcount(x)]++;
  }
  // class key (outside bits) -> member addresses
  std::map<std::pair<int, uint64_t>, std::vector<int>> classes;  // (m, key) -> members
  for (size_t i = 0; i < strs.size(); ++i) {
    uint64_t s = strs[i];
    int pat = (int)((s & wmask) >> a);
    int m = __builtin_popcount(pat);
    auto& v = classes[{m, s & ~wmask}];
    if (v.empty()) v.assign((size_t)binom(w, m), -1);
    v[prank[pat]] = (int)i;
  }
  int cur_m = -1, lane = 64;
  for (auto& kv : classes) {
    int m = kv.first.first;
    const int C = (int)binom(w, m);
    if (m != cur_m || lane == 64) {
      cur_m = m;
      lane = 0;
      t.chunk_m.push_back(m);
      t.chunk_off.push_back((int)t.tab.size());
      t.chunk_n.push_back(0);
      t.tab.resize(t.tab.size() + (size_t)C * 64, -1);
    }
    const int ch = (int)t.chunk_m.size() - 1;
    for (int k = 0; k < C; ++k) t.tab[t.chunk_off[ch] + k * 64 + lane] = kv.second[k];
    t.cls.push_back((ch << 6) | lane);
    t.chunk_n[ch] = lane + 1;
    ++lane;
  }
  return t;
}

SegWindowTable build_seg_window(const std::vector<uint64_t>& seg, int wt, int a, int w, int group) {
  SegWindowTable t;
  const uint64_t low_mask = (wt >= 64) ? ~0ull : ((1ull << wt) - 1);
  int n_low = 0;
  for (uint64_t x : seg) n_low = std::max(n_low, __builtin_popcountll(x & low_mask));
  t.nl1 = std::min(a, n_low) + 1;
  // mt(m, l, k) = sum_j C(a + pos_j, l + j) over the set bits pos_1 < ... of the k-th m-pattern
  std::vector<std::vector<int>> pats(w + 1);
  for (int x = 0; x < (1 << w); ++x) pats[__builtin_popcount(x)].push_back(x);
  const int header = (w + 1) * t.nl1;
  t.mt.assign(header, 0);
  while (t.mt.size() % 4) t.mt.push_back(0);  // tables start on 16-byte boundaries
  for (int m = 0; m <= w; ++m)
    for (int l = 0; l < t.nl1; ++l) {
      t.mt[m * t.nl1 + l] = (int)t.mt.size();
      for (int x : pats[m]) {
        int64_t v = 0;
        int j = 0;
        for (int b = 0; b < w; ++b)
          if ((x >> b) & 1) v += binom(a + b, l + (++j));
        t.mt.push_back((int)v);
      }
      while (t.mt.size() % 4) t.mt.push_back(0);
    }
  std::vector<int> prank(1 << w);
  for (int m = 0; m <= w; ++m)
    for (size_t k = 0; k < pats[m].size(); ++k) prank[pats[m][k]] = (int)k;
  const uint64_t wmask = ((1ull << w) - 1) << a;
  const uint64_t below = (1ull << a) - 1;
  struct Cls {
    int m, l, cbase, count;
  };
  std::map<std::pair<int, uint64_t>, Cls> classes;  // (m, bits outside the window) -> class
  for (size_t i = 0; i < seg.size(); ++i) {
    const uint64_t sv = seg[i] & low_mask;
    const int pat = (int)((sv & wmask) >> a);
    const int m = __builtin_popcount(pat);
    const int l = __builtin_popcountll(sv & below);
    const int off = t.mt[t.mt[m * t.nl1 + l] + prank[pat]];
    const int cbase = (int)i - off;
    auto key = std::make_pair(m, seg[i] & ~wmask);
    auto it = classes.find(key);
    if (it == classes.end()) {
      classes.emplace(key, Cls{m, l, cbase, 1});
    } else {
      if (it->second.cbase != cbase || it->second.l != l)
        throw Error(FFX_EDEVICE, "segment window table: inconsistent class base");
      ++it->second.count;
    }
  }
  // chunks of 64 classes sharing m (empty and full windows need no work)
  std::map<int, std::vector<int>> by_m;
  for (auto& kv : classes) {
    const Cls& c = kv.second;
    if (c.m == 0 || c.m == w) continue;
    if (c.count != (int)binom(w, c.m)) throw Error(FFX_EDEVICE, "segment window table: incomplete class");
    by_m[c.m].push_back((c.cbase << 5) | c.l);
  }
  // lane order: classes with the same l (whose members sit at the same
  // offsets from their bases) in groups of `group` lanes whose bases differ
  // modulo `group`, so that the lanes of one LDS access cycle hit distinct
  // banks for every member; otherwise in order of base address
  for (auto& kv : by_m) {
    std::vector<int>& v = kv.second;
    std::sort(v.begin(), v.end());
    if (group < 2) continue;
    std::map<int, std::vector<int>> by_l;
    for (int c : v) by_l[c & 31].push_back(c);
    v.clear();
    for (auto& lv : by_l) {
      std::vector<int> pool = lv.second;
      std::vector<char> taken(pool.size(), 0);
      size_t left = pool.size();
      while (left > 0) {
        std::vector<char> used(group, 0);
        int in_group = 0;
        for (size_t i = 0; i < pool.size() && in_group < group; ++i) {
          if (taken[i]) continue;
          const int slot = (pool[i] >> 5) % group;
          if (used[slot]) continue;
          used[slot] = 1;
          taken[i] = 1;
          v.push_back(pool[i]);
          ++in_group;
          --left;
        }
      }
    }
  }
  struct Chunk {
    int m;
    double cost;
    std::vector<int> codes;
  };
  std::vector<Chunk> chunks;
  for (auto& kv : by_m) {
    const int m = kv.first;
    const double cost = (double)binom(w, m) * (2.0 + (double)binom(w - 2, m - 1));
    for (size_t i = 0; i < kv.second.size(); i += 64) {
      Chunk ch{m, cost, {}};
      for (size_t j = i; j < std::min(i + 64, kv.second.size()); ++j) ch.codes.push_back(kv.second[j]);
      chunks.push_back(std::move(ch));
    }
  }
  std::stable_sort(chunks.begin(), chunks.end(), [](const Chunk& x, const Chunk& y) { return x.cost > y.cost; });
  for (auto& ch : chunks) {
    t.chunk_m.push_back(ch.m);
    for (int j = 0; j < 64; ++j) t.code.push_back(j < (int)ch.codes.size() ? ch.codes[j] : -1);
  }
  return t;
}

std::vector<std::pair<int, int>> segment_runs(const std::vector<uint64_t>& strs, int wt) {
  std::vector<std::pair<int, int>> runs;
  size_t i = 0;
  while (i < strs.size()) {
    size_t j = i;
    const uint64_t hi = wt >= 64 ? 0 : strs[i] >> wt;
    while (j < strs.size() && (wt >= 64 ? 0 : strs[j] >> wt) == hi) ++j;
    runs.push_back({(int)i, (int)(j - i)});
    i = j;
  }
  return runs;
}

std::vector<std::pair<int, int>> pack_runs(const std::vector<std::pair<int, int>>& runs, int64_t cap) {
  std::vector<std::pair<int, int>> groups;
  for (const auto& r : runs) {
    if (!groups.empty() && (int64_t)groups.back().second + r.second <= cap)
      groups.back().second += r.second;
    else
      groups.push_back(r);
  }
  return groups;
}

std::vector<CrossRange> crossing_ranges(const std::vector<uint64_t>& strs, const std::vector<std::pair<int, int>>& runs,
                                        int wt, int n) {
  std::vector<CrossRange> out(runs.size());
  std::map<uint64_t, int> by_high;
  for (size_t g = 0; g < runs.size(); ++g) by_high[strs[runs[g].first] >> wt] = (int)g;
  for (size_t g = 0; g < runs.size(); ++g) {
    const uint64_t H = strs[runs[g].first] >> wt;
    const int k = n - __builtin_popcountll(H);
    const auto it = by_high.find(H ^ 1);
    if (it == by_high.end()) continue;
    const auto& pg = runs[it->second];
    CrossRange& d = out[g];
    if (!(H & 1)) {
      if (k < 1) continue;
      d.has = true;
      d.role = 0;
      d.lo = (int)binom(wt - 1, k);
      d.cnt = (int)binom(wt - 1, k - 1);
      d.peer = pg.first;
    } else {
      d.has = true;
      d.role = 1;
      d.lo = 0;
      d.cnt = (int)binom(wt - 1, k);
      d.peer = pg.first + (int)binom(wt - 1, k + 1);
    }
    if (d.lo + d.cnt > runs[g].second || d.cnt > pg.second)
      throw Error(FFX_EDEVICE, "segment crossing ranges out of bounds");
  }
  return out;
}

void balance_seg_window(SegWindowTable& t, int w, int nwaves) {
  constexpr int kSimds = 4;
  if (nwaves < kSimds || nwaves % kSimds != 0 || t.chunk_m.empty()) return;
  const int wps = nwaves / kSimds;
  // work of one chunk in VALU issue slots for a typical stage of 10 rotations:
  // per rotation 8 per member pair plus about 10 for the broadcast and the
  // dispatch, and about 4 per member for the LDS round trip
  auto work = [&](int m) { return 10.0 * (8.0 * (double)binom(w - 2, m - 1) + 10.0) + 4.0 * (double)binom(w, m); };
  const int n = (int)t.chunk_m.size();
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(t.chunk_m[x]) > work(t.chunk_m[y]); });
  std::vector<double> load(kSimds, 0.0);
  std::vector<std::vector<int>> on(kSimds);
  for (int i : order) {
    int s = 0;
    for (int k = 1; k < kSimds; ++k)
      if (load[k] < load[s]) s = k;
    load[s] += work(t.chunk_m[i]);
    on[s].push_back(i);
  }
  // chunk j of SIMD s goes to wave s + 4 (j % wps), round j / wps
  size_t rounds = 0;
  for (int s = 0; s < kSimds; ++s) rounds = std::max(rounds, (on[s].size() + wps - 1) / wps);
  std::vector<int> slot(rounds * nwaves, -1);
  for (int s = 0; s < kSimds; ++s)
    for (size_t j = 0; j < on[s].size(); ++j)
      slot[(j / wps) * nwaves + s + kSimds * (j % wps)] = on[s][j];
  while (!slot.empty() && slot.back() < 0) slot.pop_back();
  SegWindowTable o;
  o.nl1 = t.nl1;
  o.mt = std::move(t.mt);
  for (int c : slot) {
    o.chunk_m.push_back(c < 0 ? 1 : t.chunk_m[c]);
    for (int j = 0; j < 64; ++j) o.code.push_back(c < 0 ? -1 : t.code[(size_t)c * 64 + j]);
  }
  t = std::move(o);
}

std::vector<int> pack_class_codes(const SegWindowTable& t, int mt_off) {
  std::vector<int> out(t.code.size(), -1);
  for (size_t ch = 0; ch < t.chunk_m.size(); ++ch) {
    const int m = t.chunk_m[ch];
    for (size_t l = 0; l < 64 && ch * 64 + l < t.code.size(); ++l) {
      const int c = t.code[ch * 64 + l];
      if (c < 0) continue;
      const int64_t cbase = c >> 5, moff = (int64_t)mt_off + t.mt[(size_t)m * t.nl1 + (c & 31)];
      if (cbase >= ((int64_t)1 << (31 - kCodeMoffBits)) || moff >= ((int64_t)1 << kCodeMoffBits))
        throw Error(FFX_EUNSUPPORTED, "class table exceeds the packed code fields");
      out[ch * 64 + l] = (int)((cbase << kCodeMoffBits) | moff);
    }
  }
  return out;
}

SegWindowTable replicate_seg_window(const SegWindowTable& t, int w, int R, int row_len) {
  SegWindowTable o;
  o.nl1 = t.nl1;
  o.mt = t.mt;
  std::map<int, std::vector<int>> by_m;
  for (int r = 0; r < R; ++r)
    for (size_t ch = 0; ch < t.chunk_m.size(); ++ch)
      for (int j = 0; j < 64; ++j) {
        const int c = t.code[ch * 64 + j];
        if (c < 0) continue;
        const int64_t cbase = (int64_t)(c >> 5) + (int64_t)r * row_len;
        if (cbase >= (1ll << 26)) throw Error(FFX_EUNSUPPORTED, "replicated window table too large");
        by_m[t.chunk_m[ch]].push_back((int)((cbase << 5) | (c & 31)));
      }
  for (auto& kv : by_m) std::sort(kv.second.begin(), kv.second.end());
  struct Chunk {
    int m;
    double cost;
    std::vector<int> codes;
  };
  std::vector<Chunk> chunks;
  for (auto& kv : by_m) {
    const int m = kv.first;
    const double cost = (double)binom(w, m) * (2.0 + (double)binom(w - 2, m - 1));
    for (size_t i = 0; i < kv.second.size(); i += 64) {
      Chunk ch{m, cost, {}};
      for (size_t j = i; j < std::min(i + 64, kv.second.size()); ++j) ch.codes.push_back(kv.second[j]);
      chunks.push_back(std::move(ch));
    }
  }
  std::stable_sort(chunks.begin(), chunks.end(), [](const Chunk& x, const Chunk& y) { return x.cost > y.cost; });
  for (auto& ch : chunks) {
    o.chunk_m.push_back(ch.m);
    for (int j = 0; j < 64; ++j) o.code.push_back(j < (int)ch.codes.size() ? ch.codes[j] : -1);
  }
  return o;
}

std::vector<cd> matmul(int n, const std::vector<cd>& A, const std::vector<cd>& B) {
  std::vector<cd> C((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      cd a = A[i * n + k];
      for (int j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
    }
  return C;
}

std::vector<cd> dagger(int n, const std::vector<cd>& A) {
  std::vector<cd> B((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B[j * n + i] = std::conj(A[i * n + j]);
  return B;
}

OneBodyTable build_one_body_table(int norb, const std::vector<uint64_t>& strs, const std::vector<double>& h) {
  OneBodyTable t;
  std::unordered_map<uint64_t, int32_t> addr;
  addr.reserve(strs.size() * 2);
  for (size_t i = 0; i < strs.size(); ++i) addr[strs[i]] = (int32_t)i;
  t.off.reserve(strs.size() + 1);
  t.off.push_back(0);
  for (size_t j = 0; j < strs.size(); ++j) {
    const uint64_t J = strs[j];
    double diag = 0.0;
    for (int p = 0; p < norb; ++p)
      if ((J >> p) & 1) diag += h[(size_t)p * norb + p];
    if (diag != 0.0) {
      t.src.push_back((int32_t)j);
      t.coef.push_back(diag);
    }
    // J = I - q + p with p in J, q not in J: I = J - p + q
    for (int p = 0; p < norb; ++p) {
      if (!((J >> p) & 1)) continue;
      for (int q = 0; q < norb; ++q) {
        if (q == p || ((J >> q) & 1)) continue;
        const double hv = h[(size_t)p * norb + q];
        if (hv == 0.0) continue;
        const uint64_t I = (J & ~(1ull << p)) | (1ull << q);
        const int lo = std::min(p, q), hi = std::max(p, q);
        const uint64_t between = ((1ull << hi) - 1) & ~((1ull << (lo + 1)) - 1);
        const double sign = (__builtin_popcountll(I & between) & 1) ? -1.0 : 1.0;
        auto it = addr.find(I);
        if (it == addr.end()) throw Error(FFX_EDEVICE, "one-body table: configuration not in the sector");
        t.src.push_back(it->second);
        t.coef.push_back(sign * hv);
      }
    }
    t.off.push_back((int64_t)t.src.size());
  }
  return t;
}

std::vector<double> bessel_j_series(double z, int kmax) {
  if (!(z >= 0.0) || kmax < 0) throw Error(FFX_EINVAL, "bessel_j_series: bad argument");
  std::vector<double> J((size_t)kmax + 1, 0.0);
  if (z == 0.0) {
    J[0] = 1.0;
    return J;
  }
  // start far enough above both kmax and z that the error of the arbitrary
  // starting values has decayed below double precision at k <= kmax
  const int top = std::max(kmax, (int)std::ceil(z)) + 40 + (int)std::sqrt(40.0 * (std::max(kmax, (int)z) + 1));
  const int start = top + (top & 1);
  std::vector<double> v((size_t)start + 2, 0.0);
  v[start + 1] = 0.0;
  v[start] = 1e-300;
  double norm = 0.0;
  for (int k = start; k >= 1; --k) {
    v[k - 1] = (2.0 * k / z) * v[k] - v[k + 1];
    if (std::abs(v[k - 1]) > 1e250) {  // rescale everything computed so far
      for (int j = k - 1; j <= start + 1; ++j) v[j] *= 1e-250;
      norm *= 1e-250;
    }
    if ((k - 1) % 2 == 0 && k - 1 > 0) norm += 2.0 * v[k - 1];
  }
  norm += v[0];
  for (int k = 0; k <= kmax; ++k) J[k] = v[k] / norm;
  return J;
}

void eigh(int n, const std::vector<cd>& Ain, std::vector<double>& w, std::vector<cd>& W) {
  std::vector<cd> A = Ain;
  W.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) W[i * n + i] = 1.0;
  double norm = 0;
  for (auto& x : A) norm += std::norm(x);
  norm = std::sqrt(norm);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(A[p * n + q]);
    if (std::sqrt(off) <= 1e-17 * std::max(norm, 1e-300)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        cd apq = A[p * n + q];
        double r = std::abs(apq);
        if (r == 0.0) continue;
        cd ph = apq / r;  // e^{i phi}
        double app = A[p * n + p].real(), aqq = A[q * n + q].real();
        double tau = (aqq - app) / (2 * r);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
        double c = 1 / std::sqrt(1 + t * t), s = t * c;
        // J = P R with P = diag(1, conj(ph)) on (p, q), R = [[c, s], [-s, c]]
        // columns: J[:, p] = (c, -s conj(ph)), J[:, q] = (s, c conj(ph)) in rows (p, q)
        cd jpp = c, jqp = -s * std::conj(ph), jpq = s, jqq = c * std::conj(ph);
        // A <- A J (columns)
        for (int k = 0; k < n; ++k) {
          cd x = A[k * n + p], y = A[k * n + q];
          A[k * n + p] = x * jpp + y * jqp;
          A[k * n + q] = x * jpq + y * jqq;
        }
        // A <- J^dag A (rows)
        for (int k = 0; k < n; ++k) {
          cd x = A[p * n + k], y = A[q * n + k];
          A[p * n + k] = std::conj(jpp) * x + std::conj(jqp) * y;
          A[q * n + k] = std::conj(jpq) * x + std::conj(jqq) * y;
        }
        A[p * n + q] = A[q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {
          cd x = W[k * n + p], y = W[k * n + q];
          W[k * n + p] = x * jpp + y * jqp;
          W[k * n + q] = x * jpq + y * jqq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i].real();
}

std::vector<cd> expm_antihermitian(int n, const std::vector<cd>& K) {
  // H = i K is Hermitian; K = -i H = W diag(-i w) W^dag
  std::vector<cd> H((size_t)n * n);
  for (int i = 0; i < n * n; ++i) H[i] = cd(0, 1) * K[i];
  std::vector<double> w;
  std::vector<cd> W;
  eigh(n, H, w, W);
  std::vector<cd> E((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd acc = 0;
      for (int k = 0; k < n; ++k) acc += W[i * n + k] * std::exp(cd(0, -w[k])) * std::conj(W[j * n + k]);
      E[i * n + j] = acc;
    }
  return E;
}

std::vector<cd> slater_column_minors(int norb, int n, const std::vector<cd>& U,
                                     const std::vector<uint64_t>& strs) {
  // level m: D_m(S) = det U[S, 0:m] over m-subsets S, expanded along column m-1
  std::unordered_map<uint64_t, cd> prev, cur;
  prev[0] = 1.0;
  for (int m = 1; m <= n; ++m) {
    cur.clear();
    for (uint64_t S : make_strings(norb, m)) {
      cd acc = 0;
      int i = 0;
      for (int r = 0; r < norb; ++r) {
        if (!((S >> r) & 1)) continue;
        double sign = ((i + m - 1) & 1) ? -1.0 : 1.0;
        acc += sign * U[r * norb + (m - 1)] * prev[S & ~(1ull << r)];
        ++i;
      }
      cur[S] = acc;
    }
    prev.swap(cur);
  }
  std::vector<cd> out(strs.size());
  for (size_t i = 0; i < strs.size(); ++i) out[i] = prev[strs[i]];
  return out;
}

}  // namespace ffx
