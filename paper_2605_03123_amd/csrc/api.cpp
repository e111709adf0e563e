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
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "device.h"
#include "ffx.h"
#include "host.h"

using namespace ffx;

namespace {

thread_local std::string g_last_error;

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw Error(FFX_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));          \
  } while (0)

template <class F>
int guard(F&& f) {
  try {
    g_last_error.clear();
    f();
    return FFX_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return FFX_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return FFX_EINVAL;
  }
}

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(FFX_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int d) {
    HIPCHK(hipGetDevice(&prev));
    if (prev != d) HIPCHK(hipSetDevice(d));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

std::vector<cd> load_complex(int n, const double* p) {
  std::vector<cd> v((size_t)n * n);
  for (int i = 0; i < n * n; ++i) v[i] = cd(p[2 * i], p[2 * i + 1]);
  return v;
}

std::vector<cd> load_real(int n, const double* p) {
  std::vector<cd> v((size_t)n * n);
  for (int i = 0; i < n * n; ++i) v[i] = cd(p[i], 0.0);
  return v;
}

bool all_finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct ffx_plan_s {
  int norb = 0;
  int n[2] = {0, 0};
  bool c64 = false;
  int device = 0;
  int64_t dim[2] = {0, 0};
  std::vector<uint64_t> str[2];
  uint32_t* d_masks[2] = {nullptr, nullptr};
  int W = 2;
  std::vector<dev::WinDev> win[2];
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
  double* results = nullptr;  // kResults doubles
  double* rowout = nullptr;
  std::vector<void*> allocs;
  static constexpr int kResults = 1 << 16;
  // diagnostics: event pairs around window-pass launches
  struct Timed {
    hipEvent_t a, b;
    int spin;
    double alg_bytes;
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
    if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess || !p)
      throw Error(FFX_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    allocs.push_back(p);
    return p;
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

namespace {

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
  bool committed = false;

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
    if (bytes) std::memcpy(h + off, src, bytes);
    const T* r = (const T*)(d + off);
    off += bytes;
    return r;
  }
  void commit() {
    if (off) HIPCHK(hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, s));
    committed = true;
  }
  ~Upload() { (void)hipEventRecord(P->ev[slot], s); }
};

// ---------------------------------------------------------------------------
// gate programs
// ---------------------------------------------------------------------------
struct PassProg {
  int a;
  const dev::RotDev* rots;
  int nrot;
};
struct SpinProg {
  std::vector<PassProg> passes;
  const double* delta = nullptr;
  bool has_phase = false;
  bool real = true;
};
struct RotProg {
  SpinProg sp[2];
};

SpinProg prep_spin(ffx_plan_s& P, Upload& up, const Decomposition& d) {
  SpinProg sp;
  sp.real = d.real;
  for (double x : d.phase)
    if (x != 0.0) sp.has_phase = true;
  if (sp.has_phase) sp.delta = up.put(d.phase.data(), d.phase.size());
  const int W = P.W;
  auto passes = schedule_windows(d.rots, P.norb, W);
  std::vector<dev::RotDev> buf;
  for (auto& ps : passes) {
    buf.clear();
    for (int i : ps.idx) {
      const Givens& g = d.rots[i];
      buf.push_back(dev::RotDev{g.p - ps.a, 0, g.c, g.s.real(), g.s.imag()});
    }
    sp.passes.push_back(PassProg{ps.a, up.put(buf.data(), buf.size()), (int)buf.size()});
  }
  if (sp.passes.empty() && sp.has_phase) sp.passes.push_back(PassProg{0, nullptr, 0});
  return sp;
}

RotProg prep_rotation(ffx_plan_s& P, Upload& up, const std::vector<cd>& Ua, const std::vector<cd>* Ub) {
  RotProg rp;
  Decomposition da = givens_decompose(P.norb, Ua.data());
  rp.sp[0] = prep_spin(P, up, da);
  if (Ub == nullptr) {
    rp.sp[1] = rp.sp[0];
  } else {
    Decomposition db = givens_decompose(P.norb, Ub->data());
    rp.sp[1] = prep_spin(P, up, db);
  }
  return rp;
}

void run_rotation(ffx_plan_s& P, void* vec, const RotProg& rp, hipStream_t s) {
  for (int sigma = 0; sigma < 2; ++sigma) {
    const SpinProg& sp = rp.sp[sigma];
    if (sp.has_phase) {
      dev::string_phase(P.c64, P.d_masks[sigma], P.dim[sigma], sp.delta, P.norb, P.phase_tab[sigma], s);
      check_launch();
    }
    for (size_t i = 0; i < sp.passes.size(); ++i) {
      const PassProg& pp = sp.passes[i];
      const bool last = i + 1 == sp.passes.size();
      ffx_plan_s::Timed tm{};
      if (P.timing) {
        tm.a = P.take_event();
        tm.b = P.take_event();
        tm.spin = sigma;
        const double K = 0.5 * P.norb * (P.norb - 1);
        tm.alg_bytes = K > 0 ? (pp.nrot / K) * 2.0 * (double)P.state_bytes() : 0.0;
        HIPCHK(hipEventRecord(tm.a, s));
      }
      dev::win_pass(P.c64, sp.real, sigma, vec, P.dim[0], P.dim[1], P.win[sigma][pp.a], pp.rots, pp.nrot,
                    (last && sp.has_phase) ? P.phase_tab[sigma] : nullptr, s);
      check_launch();
      if (P.timing) {
        HIPCHK(hipEventRecord(tm.b, s));
        P.timed.push_back(tm);
      }
    }
  }
}

// f(I_a, I_b) = lin_a.x_a + lin_b.x_b + 1/2 x_a Qa x_a + 1/2 x_b Qb x_b + x_a C x_b
struct DiagProg {
  dev::DiagSpecDev spec{};
  bool cross = false;
  bool has_a = false, has_b = false;
};

DiagProg prep_diag(ffx_plan_s& P, Upload& up, const double* lin_a, const double* lin_b, const double* Qa,
                   const double* Qb, const double* C) {
  const int N = P.norb;
  DiagProg d;
  if (lin_a) d.spec.lin_a = up.put(lin_a, N);
  if (lin_b) d.spec.lin_b = up.put(lin_b, N);
  if (Qa) d.spec.Qa = up.put(Qa, (size_t)N * N);
  if (Qb) d.spec.Qb = up.put(Qb, (size_t)N * N);
  if (C) {
    d.spec.C = up.put(C, (size_t)N * N);
    d.cross = true;
  }
  d.has_a = lin_a || Qa;
  d.has_b = lin_b || Qb;
  return d;
}

dev::DiagDev build_diag(ffx_plan_s& P, const DiagProg& d, hipStream_t s) {
  dev::diag_tables(P.d_masks[0], P.dim[0], P.d_masks[1], P.dim[1], P.norb, d.spec, d.has_a ? P.dA : nullptr,
                   d.has_b ? P.dB : nullptr, d.cross ? P.dV : nullptr, s);
  check_launch();
  return dev::DiagDev{d.has_a ? P.dA : nullptr, d.has_b ? P.dB : nullptr, d.cross ? P.dV : nullptr};
}

void run_diag_phase(ffx_plan_s& P, void* vec, const DiagProg& d, double scale, hipStream_t s) {
  dev::DiagDev f = build_diag(P, d, s);
  dev::diag_phase(P.c64, vec, P.dim[0], P.dim[1], P.d_masks[0], P.norb, f, scale, s);
  check_launch();
}

// ---------------------------------------------------------------------------
// DF Hamiltonian data on the host
// ---------------------------------------------------------------------------
struct DFHost {
  int L = 0;
  std::vector<double> eps;          // eigenvalues of h
  std::vector<cd> V;                // eigenvectors of h (columns)
  std::vector<std::vector<cd>> U;   // U_t
  std::vector<std::vector<double>> J;
  // W_0 = V, W_t = U_t
  const std::vector<cd>& Wm(int term) const { return term == 0 ? V : U[term - 1]; }
};

DFHost load_df(const ffx_plan_s& P, const ffx_df_ham* ham) {
  if (!ham || !ham->h || (ham->n_terms > 0 && (!ham->J || !ham->U)))
    throw Error(FFX_EINVAL, "DF Hamiltonian has a null pointer");
  if (ham->norb != P.norb) throw Error(FFX_EINVAL, "DF Hamiltonian norb does not match the plan");
  if (ham->n_terms < 0) throw Error(FFX_EINVAL, "negative n_terms");
  const int N = P.norb;
  DFHost d;
  d.L = ham->n_terms;
  if (!all_finite(ham->h, (size_t)N * N)) throw Error(FFX_EINVAL, "non-finite h");
  std::vector<cd> h = load_real(N, ham->h);
  eigh(N, h, d.eps, d.V);
  // h is real symmetric: make the eigenvectors real (a real phase choice per column)
  for (int j = 0; j < N; ++j) {
    int big = 0;
    for (int i = 1; i < N; ++i)
      if (std::abs(d.V[i * N + j]) > std::abs(d.V[big * N + j])) big = i;
    cd ph = std::abs(d.V[big * N + j]) > 0 ? std::conj(d.V[big * N + j]) / std::abs(d.V[big * N + j]) : 1.0;
    for (int i = 0; i < N; ++i) d.V[i * N + j] = cd((d.V[i * N + j] * ph).real(), 0.0);
  }
  // re-orthonormalise (Gram-Schmidt in FP64) to remove rounding from the phase fix
  for (int j = 0; j < N; ++j) {
    for (int k = 0; k < j; ++k) {
      double dot = 0;
      for (int i = 0; i < N; ++i) dot += d.V[i * N + j].real() * d.V[i * N + k].real();
      for (int i = 0; i < N; ++i) d.V[i * N + j] -= dot * d.V[i * N + k];
    }
    double nr = 0;
    for (int i = 0; i < N; ++i) nr += std::norm(d.V[i * N + j]);
    nr = std::sqrt(nr);
    for (int i = 0; i < N; ++i) d.V[i * N + j] /= nr;
  }
  for (int t = 0; t < d.L; ++t) {
    if (!all_finite(ham->J + (size_t)t * N * N, (size_t)N * N) || !all_finite(ham->U + (size_t)2 * t * N * N, (size_t)2 * N * N))
      throw Error(FFX_EINVAL, "non-finite DF term");
    d.U.push_back(load_complex(N, ham->U + (size_t)2 * t * N * N));
    d.J.emplace_back(ham->J + (size_t)t * N * N, ham->J + (size_t)(t + 1) * N * N);
  }
  return d;
}

DiagProg prep_df_weight(ffx_plan_s& P, Upload& up, const DFHost& df, int term) {
  if (term == 0) return prep_diag(P, up, df.eps.data(), df.eps.data(), nullptr, nullptr, nullptr);
  const double* J = df.J[term - 1].data();
  return prep_diag(P, up, nullptr, nullptr, J, J, J);
}

// product formula as a list of (term, time) in application order
void product_formula(int order, double t, int n_terms_total, std::vector<std::pair<int, double>>& out) {
  if (order == 0) {
    for (int k = 0; k < n_terms_total; ++k) out.push_back({k, t});
  } else if (order == 1) {
    for (int k = 0; k < n_terms_total; ++k) out.push_back({k, t / 2});
    for (int k = n_terms_total - 1; k >= 0; --k) out.push_back({k, t / 2});
  } else {
    double u = 1.0 / (4.0 - std::pow(4.0, 1.0 / (2 * order - 1)));
    for (double tau : {u * t, u * t, (1 - 4 * u) * t, u * t, u * t}) product_formula(order - 1, tau, n_terms_total, out);
  }
}

// LUCJ parameters on the host
struct LUCJHost {
  int R = 0;
  std::vector<std::vector<cd>> K, U;
  std::vector<std::vector<double>> Jsame, Jopp;
};

LUCJHost load_lucj(const ffx_plan_s& P, const ffx_lucj* op) {
  if (!op || !op->params) throw Error(FFX_EINVAL, "LUCJ operator has a null pointer");
  if (op->norb != P.norb) throw Error(FFX_EINVAL, "LUCJ norb does not match the plan");
  if (op->n_reps < 1) throw Error(FFX_EINVAL, "n_reps must be >= 1");
  const int N = P.norb;
  const int per = 2 * N * N + 2 * N - 1;
  if (!all_finite(op->params, (size_t)per * op->n_reps)) throw Error(FFX_EINVAL, "non-finite LUCJ parameter");
  LUCJHost L;
  L.R = op->n_reps;
  for (int k = 0; k < L.R; ++k) {
    const double* th = op->params + (size_t)k * per;
    std::vector<cd> A((size_t)N * N), K((size_t)N * N);
    for (int i = 0; i < N * N; ++i) A[i] = cd(th[i], th[N * N + i]);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) K[i * N + j] = A[i * N + j] - std::conj(A[j * N + i]);
    std::vector<double> Js((size_t)N * N, 0.0), Jo((size_t)N * N, 0.0);
    for (int p = 0; p + 1 < N; ++p) Js[p * N + p + 1] = Js[(p + 1) * N + p] = th[2 * N * N + p];
    for (int p = 0; p < N; ++p) Jo[p * N + p] = th[2 * N * N + N - 1 + p];
    L.U.push_back(expm_antihermitian(N, K));
    L.K.push_back(std::move(K));
    L.Jsame.push_back(std::move(Js));
    L.Jopp.push_back(std::move(Jo));
  }
  return L;
}

struct LUCJProg {
  std::vector<RotProg> after;   // after[k]: rotation after D_k (U_{k+1}^dag U_k, or U_R)
  std::vector<RotProg> undo;    // inverse of after[k]
  std::vector<DiagProg> diag;   // D_k
  const double* a = nullptr;    // Slater vectors (complex, interleaved)
  const double* b = nullptr;
};

LUCJProg prep_lucj(ffx_plan_s& P, Upload& up, const LUCJHost& L, bool with_inverse) {
  const int N = P.norb;
  LUCJProg g;
  std::vector<cd> U1d = dagger(N, L.U[0]);
  auto sa = slater_column_minors(N, P.n[0], U1d, P.str[0]);
  auto sb = (P.n[1] == P.n[0]) ? sa : slater_column_minors(N, P.n[1], U1d, P.str[1]);
  g.a = up.put((const double*)sa.data(), 2 * sa.size());
  g.b = up.put((const double*)sb.data(), 2 * sb.size());
  for (int k = 0; k < L.R; ++k) {
    std::vector<cd> M = (k + 1 < L.R) ? matmul(N, dagger(N, L.U[k + 1]), L.U[k]) : L.U[k];
    g.after.push_back(prep_rotation(P, up, M, nullptr));
    if (with_inverse) g.undo.push_back(prep_rotation(P, up, dagger(N, M), nullptr));
    g.diag.push_back(prep_diag(P, up, nullptr, nullptr, L.Jsame[k].data(), L.Jsame[k].data(), L.Jopp[k].data()));
  }
  return g;
}

void run_lucj_forward(ffx_plan_s& P, void* vec, const LUCJProg& g, int R, hipStream_t s) {
  dev::outer(P.c64, g.a, g.b, vec, P.dim[0], P.dim[1], s);
  check_launch();
  for (int k = 0; k < R; ++k) {
    run_diag_phase(P, vec, g.diag[k], -1.0, s);
    run_rotation(P, vec, g.after[k], s);
  }
}

void validate_plan(ffx_plan plan) {
  if (!plan) throw Error(FFX_EINVAL, "null plan");
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// Gradient with respect to A (K = A - A^dag, U = expm(K)) given G such that
// dE = 2 Re sum_pq (U^dag dU)_pq G_pq, via the adjoint of the Frechet
// derivative of expm at the anti-Hermitian K = W diag(-i w) W^dag.
void expm_param_grad(int N, const std::vector<cd>& K, const std::vector<cd>& G, double* g_re, double* g_im) {
  std::vector<cd> H((size_t)N * N);
  for (int i = 0; i < N * N; ++i) H[i] = cd(0, 1) * K[i];
  std::vector<double> w;
  std::vector<cd> W;
  eigh(N, H, w, W);
  // Q_ij = e^{+i w_i} (W^T G W^*)_ij ; Phi_ij = e^{-i (w_i + w_j)/2} sinc((w_i - w_j)/2)
  std::vector<cd> WT((size_t)N * N), Wc((size_t)N * N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      WT[i * N + j] = W[j * N + i];
      Wc[i * N + j] = std::conj(W[i * N + j]);
    }
  std::vector<cd> Q = matmul(N, matmul(N, WT, G), Wc);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double d = 0.5 * (w[i] - w[j]);
      double sinc = std::fabs(d) < 1e-8 ? 1.0 - d * d / 6.0 : std::sin(d) / d;
      cd phi = std::exp(cd(0, -0.5 * (w[i] + w[j]))) * sinc;
      Q[i * N + j] *= std::exp(cd(0, w[i])) * phi;
    }
  // Z = W^* R W^T
  std::vector<cd> Z = matmul(N, matmul(N, Wc, Q), WT);
  for (int p = 0; p < N; ++p)
    for (int q = 0; q < N; ++q) {
      g_re[p * N + q] = 2.0 * (Z[p * N + q] - Z[q * N + p]).real();
      g_im[p * N + q] = 2.0 * (cd(0, 1) * (Z[p * N + q] + Z[q * N + p])).real();
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// exported API
// ---------------------------------------------------------------------------
extern "C" {

const char* ffx_last_error(void) { return g_last_error.c_str(); }

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
    if (hipHostMalloc((void**)&P->h_ring, P->slot_bytes * ffx_plan_s::kSlots, hipHostMallocDefault) != hipSuccess)
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
    P->rowout = (double*)P->dalloc((size_t)dmax * 2 * norb * 8);
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

int ffx_apply_orbital_rotation(ffx_plan plan, void* vec, const double* U_a, const double* U_b, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !U_a) throw Error(FFX_EINVAL, "null vec or U_a");
    const int N = plan->norb;
    if (!all_finite(U_a, (size_t)2 * N * N) || (U_b && !all_finite(U_b, (size_t)2 * N * N)))
      throw Error(FFX_EINVAL, "non-finite U");
    DeviceGuard dg(plan->device);
    hipStream_t s = as_stream(stream);
    auto Ua = load_complex(N, U_a);
    std::vector<cd> Ub;
    if (U_b) Ub = load_complex(N, U_b);
    Upload up(plan, s);
    RotProg rp = prep_rotation(*plan, up, Ua, U_b ? &Ub : nullptr);
    up.commit();
    run_rotation(*plan, vec, rp, s);
  });
}

int ffx_apply_num_op_sum_evolution(ffx_plan plan, void* vec, const double* lam_a, const double* lam_b,
                                   double time, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !lam_a) throw Error(FFX_EINVAL, "null vec or lam_a");
    const int N = plan->norb;
    if (!std::isfinite(time) || !all_finite(lam_a, N) || (lam_b && !all_finite(lam_b, N)))
      throw Error(FFX_EINVAL, "non-finite parameter");
    DeviceGuard dg(plan->device);
    hipStream_t s = as_stream(stream);
    Upload up(plan, s);
    DiagProg d = prep_diag(*plan, up, lam_a, lam_b ? lam_b : lam_a, nullptr, nullptr, nullptr);
    up.commit();
    run_diag_phase(*plan, vec, d, -time, s);
  });
}

int ffx_apply_diag_coulomb_evolution(ffx_plan plan, void* vec, const double* J_aa, const double* J_ab,
                                     const double* J_bb, double time, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!vec || !J_aa) throw Error(FFX_EINVAL, "null vec or J_aa");
    const int N = plan->norb;
    const double* Jab = J_ab ? J_ab : J_aa;
    const double* Jbb = J_bb ? J_bb : J_aa;
    if (!std::isfinite(time) || !all_finite(J_aa, (size_t)N * N) || !all_finite(Jab, (size_t)N * N) ||
        !all_finite(Jbb, (size_t)N * N))
      throw Error(FFX_EINVAL, "non-finite parameter");
    DeviceGuard dg(plan->device);
    hipStream_t s = as_stream(stream);
    Upload up(plan, s);
    DiagProg d = prep_diag(*plan, up, nullptr, nullptr, J_aa, Jbb, Jab);
    up.commit();
    run_diag_phase(*plan, vec, d, -time, s);
  });
}

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
    Upload up(&P, s);
    std::map<std::pair<int, int>, RotProg> rot_cache;
    auto rot = [&](int from, int to) -> const RotProg& {
      auto key = std::make_pair(from, to);
      auto it = rot_cache.find(key);
      if (it != rot_cache.end()) return it->second;
      std::vector<cd> M;
      if (from < 0)
        M = dagger(N, df.Wm(to));
      else if (to < 0)
        M = df.Wm(from);
      else
        M = matmul(N, dagger(N, df.Wm(to)), df.Wm(from));
      return rot_cache.emplace(key, prep_rotation(P, up, M, nullptr)).first->second;
    };
    std::vector<DiagProg> weights;
    for (int t = 0; t <= df.L; ++t) weights.push_back(prep_df_weight(P, up, df, t));
    // prepare every rotation before the upload is committed
    int prev = -1;
    for (auto& e : m) {
      rot(prev, e.first);
      prev = e.first;
    }
    rot(prev, -1);
    up.commit();
    prev = -1;
    for (auto& e : m) {
      run_rotation(P, vec, rot(prev, e.first), s);
      run_diag_phase(P, vec, weights[e.first], -e.second, s);
      prev = e.first;
    }
    run_rotation(P, vec, rot(prev, -1), s);
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
    Upload up(&P, s);
    LUCJProg g = prep_lucj(P, up, L, false);
    up.commit();
    run_lucj_forward(P, vec, g, L.R, s);
  });
}

int64_t ffx_workspace_bytes(ffx_plan plan, int what) {
  if (!plan) return -1;
  const int64_t S = ((int64_t)plan->state_bytes() + 255) / 256 * 256;
  if (what == 0) return S;
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
    Upload up(&P, s);
    std::vector<RotProg> rots;
    std::vector<DiagProg> w;
    for (int t = 0; t <= df.L; ++t) {
      rots.push_back(prep_rotation(P, up, dagger(N, df.Wm(t)), nullptr));
      w.push_back(prep_df_weight(P, up, df, t));
    }
    up.commit();
    for (int t = 0; t <= df.L; ++t) {
      HIPCHK(hipMemcpyAsync(tmp, vec, P.state_bytes(), hipMemcpyDeviceToDevice, s));
      run_rotation(P, tmp, rots[t], s);
      dev::DiagDev f = build_diag(P, w[t], s);
      int np = dev::diag_expect(P.c64, tmp, P.dim[0], P.dim[1], P.d_masks[0], N, f, P.partials, s);
      dev::sum_partials(P.partials, np, P.results + t, s);
      check_launch();
    }
    std::vector<double> r(df.L + 1);
    HIPCHK(hipMemcpyAsync(r.data(), P.results, r.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double e = 0;
    for (double x : r) e += x;
    *energy = e;
  });
}

int ffx_lucj_energy_grad(ffx_plan plan, const ffx_lucj* op, const ffx_df_ham* ham, double* energy, double* grad,
                         void* psi_out, void* workspace, void* stream) {
  return guard([&] {
    validate_plan(plan);
    if (!energy || !grad || !workspace) throw Error(FFX_EINVAL, "null pointer");
    ffx_plan_s& P = *plan;
    const int N = P.norb;
    LUCJHost L = load_lucj(P, op);
    DFHost df = load_df(P, ham);
    DeviceGuard dg(P.device);
    hipStream_t s = as_stream(stream);
    const size_t S = P.state_bytes();
    const size_t Sa = (S + 255) / 256 * 256;
    char* ws = (char*)workspace;
    void* lam = ws;
    void* tmp = ws + Sa;
    void* psiT = ws + 2 * Sa;
    void* lamT = ws + 3 * Sa;
    void* psi = psi_out ? psi_out : (void*)(ws + 4 * Sa);
    double* part = (double*)(ws + 5 * Sa);
    Upload up(&P, s);
    LUCJProg g = prep_lucj(P, up, L, true);
    std::vector<RotProg> to_t, from_t;
    std::vector<DiagProg> w;
    for (int t = 0; t <= df.L; ++t) {
      to_t.push_back(prep_rotation(P, up, dagger(N, df.Wm(t)), nullptr));
      from_t.push_back(prep_rotation(P, up, df.Wm(t), nullptr));
      w.push_back(prep_df_weight(P, up, df, t));
    }
    up.commit();
    // forward
    run_lucj_forward(P, psi, g, L.R, s);
    // costate lambda = H psi = sum_t U_t D_t U_t^dag psi
    for (int t = 0; t <= df.L; ++t) {
      void* dst = (t == 0) ? lam : tmp;
      HIPCHK(hipMemcpyAsync(dst, psi, S, hipMemcpyDeviceToDevice, s));
      run_rotation(P, dst, to_t[t], s);
      dev::DiagDev f = build_diag(P, w[t], s);
      dev::diag_scale(P.c64, dst, P.dim[0], P.dim[1], P.d_masks[0], N, f, s);
      check_launch();
      run_rotation(P, dst, from_t[t], s);
      if (t > 0) {
        dev::axpy(P.c64, tmp, lam, P.elems(), s);
        check_launch();
      }
    }
    // energy <psi|lambda>
    dev::inner(P.c64, psi, lam, P.elems(), P.partials, P.results, s);
    check_launch();
    // reverse sweep: uncompute psi and lambda, collecting transition matrices
    const int NN = N * N;
    double* Tdev = P.results + 16;                       // per rep: T_b (alpha, beta), T_a (alpha, beta)
    double* Ddev = P.results + 16 + (size_t)L.R * 8 * NN;  // per rep: 2N-1 diagonal-gate gradients
    if (16 + (size_t)L.R * (8 * NN + 2 * N) > (size_t)ffx_plan_s::kResults)
      throw Error(FFX_EUNSUPPORTED, "too many LUCJ repetitions for the result buffer");
    auto rdm = [&](double* Tout) {
      dev::rdm_rows(P.c64, lam, psi, P.dim[0], P.dim[1], P.d_masks[0], N, part, s);
      dev::rdm_reduce(part, P.dim[0], N, Tout, s);
      dev::transpose(P.c64, psi, psiT, P.dim[0], P.dim[1], s);
      dev::transpose(P.c64, lam, lamT, P.dim[0], P.dim[1], s);
      dev::rdm_rows(P.c64, lamT, psiT, P.dim[1], P.dim[0], P.d_masks[1], N, part, s);
      dev::rdm_reduce(part, P.dim[1], N, Tout + 2 * NN, s);
      check_launch();
    };
    for (int k = L.R - 1; k >= 0; --k) {
      run_rotation(P, psi, g.undo[k], s);
      run_rotation(P, lam, g.undo[k], s);
      rdm(Tdev + (size_t)k * 8 * NN);
      dev::diag_grad_rows(P.c64, lam, psi, P.dim[0], P.dim[1], P.d_masks[1], N, P.rowout, s);
      dev::diag_grad_combine(P.rowout, P.dim[0], P.d_masks[0], N, Ddev + (size_t)k * (2 * N), s);
      check_launch();
      run_diag_phase(P, psi, g.diag[k], +1.0, s);
      run_diag_phase(P, lam, g.diag[k], +1.0, s);
      rdm(Tdev + (size_t)k * 8 * NN + 4 * NN);
    }
    std::vector<double> res(16 + (size_t)L.R * (8 * NN + 2 * N));
    HIPCHK(hipMemcpyAsync(res.data(), P.results, res.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *energy = res[0];
    const int per = 2 * NN + 2 * N - 1;
    for (int k = 0; k < L.R; ++k) {
      const double* Tb = res.data() + 16 + (size_t)k * 8 * NN;
      const double* Ta = Tb + 4 * NN;
      std::vector<cd> G((size_t)NN);
      for (int i = 0; i < NN; ++i)
        G[i] = cd(Tb[2 * i] + Tb[2 * NN + 2 * i] - Ta[2 * i] - Ta[2 * NN + 2 * i],
                  Tb[2 * i + 1] + Tb[2 * NN + 2 * i + 1] - Ta[2 * i + 1] - Ta[2 * NN + 2 * i + 1]);
      double* gk = grad + (size_t)k * per;
      expm_param_grad(N, L.K[k], G, gk, gk + NN);
      const double* dg = res.data() + 16 + (size_t)L.R * 8 * NN + (size_t)k * (2 * N);
      for (int i = 0; i < 2 * N - 1; ++i) gk[2 * NN + i] = dg[i];
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

int ffx_timing_read(ffx_plan plan, int spin, double* total_ms, int64_t* launches, double* alg_bytes) {
  return guard([&] {
    validate_plan(plan);
    if (spin != 0 && spin != 1) throw Error(FFX_EINVAL, "bad spin");
    DeviceGuard dg(plan->device);
    double ms = 0, bytes = 0;
    int64_t n = 0;
    for (auto& t : plan->timed) {
      if (t.spin != spin) continue;
      HIPCHK(hipEventSynchronize(t.b));
      float e = 0;
      HIPCHK(hipEventElapsedTime(&e, t.a, t.b));
      ms += e;
      bytes += t.alg_bytes;
      ++n;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    if (alg_bytes) *alg_bytes = bytes;
  });
}

}  // extern "C"
