// Internal: host-side drivers shared by the single-instance and batched entry
// points: loading of DF Hamiltonians and LUCJ parameters, Givens
// decompositions kept for the duration of a call, the LUCJ gate programs, the
// chain rule of the adjoint gradient through U = expm(K), and the error guard
// of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <deque>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "ffx.h"
#include "host.h"
#include "plan.h"

namespace ffx {

// message of the last failure on this thread
std::string& last_error();

template <class F>
int guard(F&& f) {
  try {
    last_error().clear();
    f();
    return FFX_OK;
  } catch (const Error& e) {
    last_error() = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    last_error() = "host allocation failed";
    return FFX_ENOMEM;
  } catch (const std::exception& e) {
    last_error() = e.what();
    return FFX_EINVAL;
  }
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

// ---------------------------------------------------------------------------
// Givens decompositions kept alive for the duration of one call
// ---------------------------------------------------------------------------
struct DecompPool {
  std::deque<Decomposition> v;
  const Decomposition* add(int N, const std::vector<cd>& U) {
    v.push_back(givens_decompose(N, U.data()));
    return &v.back();
  }
};

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

// LUCJ parameters on the host
struct LUCJHost {
  int R = 0;
  std::vector<std::vector<cd>> K, U;
  std::vector<std::vector<double>> Jsame, Jopp;
};

// Slater column minors of U_1^dag and the merged rotations of the ansatz:
// after[k] = U_{k+1}^dag U_k (k < R-1), after[R-1] = U_R; undo[k] = after[k]^dag.
struct LUCJParts {
  std::vector<cd> a, b;
  std::vector<const Decomposition*> after, undo;
  std::vector<DiagSpec> diag;
};

std::vector<cd> load_complex(int n, const double* p);

std::vector<cd> load_real(int n, const double* p);

bool all_finite(const double* p, size_t n);

DFHost load_df(const ffx_plan_s& P, const ffx_df_ham* ham);

// term 0: sum_p eps_p N_p (one-body term in the eigenbasis of h);
// term t: 1/2 sum_pq J_t[p][q] N_p N_q
DiagSpec df_weight_spec(const DFHost& df, int term);

// The terms of H = sum_t script-U(W_t) D_t script-U(W_t)^dag as gate programs
// (W_0 = V with D_0 = sum_p eps_p N_p, W_t = U_t with D_t = 1/2 sum_pq J_t N_p N_q):
// rotate into the term's basis, scale by its diagonal weight, rotate back.
std::vector<Program> df_term_programs(const DFHost& df, DecompPool& pool, int N);

// An interval [lo, hi] holding every eigenvalue of the DF Hamiltonian in the
// (na, nb) sector: the sum over terms of the range of each diagonal weight
// (exact for the one-body term; for a two-body term the eigenvalue range of
// J_t times the range of |x|^2, x = occupation-number vector of both spins).
void df_spectrum_bounds(const DFHost& df, int N, int na, int nb, double* lo, double* hi);

// product formula as a list of (term, time) in application order
void product_formula(int order, double t, int n_terms_total, std::vector<std::pair<int, double>>& out);

LUCJHost load_lucj(const ffx_plan_s& P, const ffx_lucj* op);

LUCJParts lucj_parts(const ffx_plan_s& P, const LUCJHost& L, DecompPool& pool, bool with_inverse);

// D_1, rotation, D_2, rotation, ... applied to the Slater determinant
Program lucj_forward_program(const LUCJParts& g, int R);

// Gradient with respect to A (K = A - A^dag, U = expm(K)) given G such that
// dE = 2 Re sum_pq (U^dag dU)_pq G_pq, via the adjoint of the Frechet
// derivative of expm at the anti-Hermitian K = W diag(-i w) W^dag.
void expm_param_grad(int N, const std::vector<cd>& K, const std::vector<cd>& G, double* g_re, double* g_im);

// Everything the LUCJ energy and its adjoint gradient run, as gate programs:
//   fwd          the ansatz applied to the Slater determinant a b^T
//   terms[t]     U_t D_t U_t^dag (t = 0: the one-body term), summed into the
//                costate lambda = H psi
//   undo_rot[k]  the inverse of the k-th merged rotation (reverse sweep, on
//                psi and on lambda)
//   undo_diag[k] the inverse of the k-th diagonal gate
struct LUCJGrad {
  LUCJHost L;
  DFHost df;
  DecompPool pool;
  LUCJParts g;
  Program fwd;
  std::vector<Program> terms, undo_rot, undo_diag;
};
std::unique_ptr<LUCJGrad> build_lucj_grad(const ffx_plan_s& P, const ffx_lucj* op, const ffx_df_ham* ham);

// Gradient of one instance from the reverse sweep's reductions, per rep k:
// Tb[k], Ta[k] = transition one-body matrices <lambda| sum_sigma a+_p a_q |psi>
// (complex, row-major, both spins summed) before and after the diagonal gate,
// D[k] = the 2N-1 diagonal-gate gradients.  grad has n_reps (2N^2 + 2N - 1) entries.
void lucj_grad_assemble(const LUCJGrad& G, int N, const std::vector<const double*>& Tb,
                        const std::vector<const double*>& Ta, const std::vector<const double*>& D, double* grad);

}  // namespace ffx
