// Host-side drivers shared by the single-instance and batched entry points.
#include "drivers.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

namespace ffx {

std::string& last_error() {
  thread_local std::string msg;
  return msg;
}

bool fault_hit(const char* site) {
  static std::mutex mu;
  static std::string armed;
  static long long calls = 0;
  std::lock_guard<std::mutex> lock(mu);
  const char* e = std::getenv("FFX_FAULT");
  if (!e || !*e) {
    armed.clear();
    calls = 0;
    return false;
  }
  if (armed != e) {
    armed = e;
    calls = 0;
  }
  const char* colon = std::strchr(e, ':');
  if (!colon || std::strncmp(e, site, (size_t)(colon - e)) != 0 || site[colon - e] != '\0') return false;
  const long long k = std::atoll(colon + 1);
  return k >= 1 && ++calls == k;
}

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

// term 0: sum_p eps_p N_p (one-body term in the eigenbasis of h);
// term t: 1/2 sum_pq J_t[p][q] N_p N_q
DiagSpec df_weight_spec(const DFHost& df, int term) {
  DiagSpec d;
  if (term == 0) {
    d.lin_a = d.lin_b = df.eps.data();
  } else {
    const double* J = df.J[term - 1].data();
    d.Qa = d.Qb = d.C = J;
  }
  return d;
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

LUCJParts lucj_parts(const ffx_plan_s& P, const LUCJHost& L, DecompPool& pool, bool with_inverse) {
  const int N = P.norb;
  LUCJParts g;
  std::vector<cd> U1d = dagger(N, L.U[0]);
  g.a = slater_column_minors(N, P.n[0], U1d, P.str[0]);
  g.b = (P.n[1] == P.n[0]) ? g.a : slater_column_minors(N, P.n[1], U1d, P.str[1]);
  for (int k = 0; k < L.R; ++k) {
    std::vector<cd> M = (k + 1 < L.R) ? matmul(N, dagger(N, L.U[k + 1]), L.U[k]) : L.U[k];
    g.after.push_back(pool.add(N, M));
    if (with_inverse) g.undo.push_back(pool.add(N, dagger(N, M)));
    DiagSpec d;
    d.Qa = d.Qb = L.Jsame[k].data();
    d.C = L.Jopp[k].data();
    g.diag.push_back(d);
  }
  return g;
}

// D_1, rotation, D_2, rotation, ... applied to the Slater determinant
Program lucj_forward_program(const LUCJParts& g, int R) {
  Program pr;
  for (int k = 0; k < R; ++k) {
    int d = pr.add_diag(g.diag[k]);
    pr.phase(d, -1.0);
    pr.rot(g.after[k], g.after[k]);
  }
  return pr;
}

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

std::vector<Program> df_term_programs(const DFHost& df, DecompPool& pool, int N) {
  std::vector<Program> terms(df.L + 1);
  for (int t = 0; t <= df.L; ++t) {
    const Decomposition* to = pool.add(N, dagger(N, df.Wm(t)));
    const Decomposition* from = pool.add(N, df.Wm(t));
    terms[t].rot(to, to);
    terms[t].scale(terms[t].add_diag(df_weight_spec(df, t)));
    terms[t].rot(from, from);
  }
  return terms;
}

void df_spectrum_bounds(const DFHost& df, int N, int na, int nb, double* lo, double* hi) {
  std::vector<double> e = df.eps;
  std::sort(e.begin(), e.end());
  double l = 0, h = 0;
  for (int k = 0; k < na; ++k) l += e[k], h += e[N - 1 - k];
  for (int k = 0; k < nb; ++k) l += e[k], h += e[N - 1 - k];
  // |x|^2 = na + nb + 2 (doubly occupied orbitals)
  const double x2min = na + nb + 2.0 * std::max(0, na + nb - N);
  const double x2max = na + nb + 2.0 * std::min(na, nb);
  for (int t = 0; t < df.L; ++t) {
    std::vector<cd> Jc((size_t)N * N);
    for (int i = 0; i < N * N; ++i) Jc[i] = df.J[t][i];
    std::vector<double> w;
    std::vector<cd> W;
    eigh(N, Jc, w, W);
    const double wmin = *std::min_element(w.begin(), w.end());
    const double wmax = *std::max_element(w.begin(), w.end());
    l += 0.5 * std::min(wmin * x2min, wmin * x2max);
    h += 0.5 * std::max(wmax * x2min, wmax * x2max);
  }
  *lo = l;
  *hi = h;
}

std::unique_ptr<LUCJGrad> build_lucj_grad(const ffx_plan_s& P, const ffx_lucj* op, const ffx_df_ham* ham) {
  const int N = P.norb;
  auto G = std::make_unique<LUCJGrad>();
  G->L = load_lucj(P, op);
  G->df = load_df(P, ham);
  G->g = lucj_parts(P, G->L, G->pool, true);
  G->fwd = lucj_forward_program(G->g, G->L.R);
  G->terms = df_term_programs(G->df, G->pool, N);
  G->undo_rot.resize(G->L.R);
  G->undo_diag.resize(G->L.R);
  for (int k = 0; k < G->L.R; ++k) {
    G->undo_rot[k].rot(G->g.undo[k], G->g.undo[k]);
    G->undo_diag[k].phase(G->undo_diag[k].add_diag(G->g.diag[k]), +1.0);
  }
  return G;
}

void lucj_grad_assemble(const LUCJGrad& G, int N, const std::vector<const double*>& Tb,
                        const std::vector<const double*>& Ta, const std::vector<const double*>& D, double* grad) {
  const int NN = N * N;
  const int per = 2 * NN + 2 * N - 1;
  for (int k = 0; k < G.L.R; ++k) {
    std::vector<cd> M((size_t)NN);
    for (int i = 0; i < NN; ++i)
      M[i] = cd(Tb[k][2 * i] - Ta[k][2 * i], Tb[k][2 * i + 1] - Ta[k][2 * i + 1]);
    double* gk = grad + (size_t)k * per;
    expm_param_grad(N, G.L.K[k], M, gk, gk + NN);
    for (int i = 0; i < 2 * N - 1; ++i) gk[2 * NN + i] = D[k][i];
  }
}

}  // namespace ffx
