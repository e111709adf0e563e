// C ABI: the remaining gates of Table 1 (number and number-number
// interactions, Givens rotation, tunneling interaction, quadratic Hamiltonian
// evolution), the Slater-determinant state (Sec. 2.4) and the unitary cluster
// Jastrow forward pass with per-spin rotations and full diagonal-Coulomb
// matrices (Sec. 4.5.1).  Each is a gate program on the kernels of the
// orbital-rotation and diagonal passes; this file only prepares FP64 host data.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "device.h"
#include "drivers.h"
#include "ffx.h"
#include "host.h"
#include "plan.h"

using namespace ffx;

namespace {

std::vector<cd> identity(int N) {
  std::vector<cd> I((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i) I[i * N + i] = 1.0;
  return I;
}

void check_orbital(const ffx_plan_s& P, int p, const char* what) {
  if (p < 0 || p >= P.norb) throw Error(FFX_EINVAL, std::string(what) + ": orbital index out of range");
}

void check_spin(int spin) {
  if (spin != 0 && spin != 1) throw Error(FFX_EINVAL, "spin must be 0 (alpha) or 1 (beta)");
}

// compile and run one program in place on vec
void run_program(ffx_plan_s& P, const Program& pr, void* vec, void* stream) {
  DeviceGuard dg(P.device);
  hipStream_t s = (hipStream_t)stream;
  Upload up(&P, s);
  Compiled c = compile_program(P, up, pr, FINAL_STORE, s);
  up.commit();
  execute_program(P, c, vec, vec, nullptr, s);
}

// U on one spin, the identity on the other (identity decompositions drop out
// of the program)
void rotate_one_spin(ffx_plan_s& P, void* vec, const std::vector<cd>& U, int spin, void* stream) {
  const int N = P.norb;
  DecompPool pool;
  const Decomposition* du = pool.add(N, U);
  const Decomposition* di = pool.add(N, identity(N));
  Program pr;
  if (spin == 0)
    pr.rot(du, di);
  else
    pr.rot(di, du);
  run_program(P, pr, vec, stream);
}

}  // namespace

int ffx_apply_num_interaction(ffx_plan plan, void* vec, double theta, int p, int spin, void* stream) {
  return guard([&] {
    if (!plan || !vec) throw Error(FFX_EINVAL, "null plan or vec");
    if (!std::isfinite(theta)) throw Error(FFX_EINVAL, "non-finite theta");
    check_orbital(*plan, p, "number interaction");
    check_spin(spin);
    const int N = plan->norb;
    // exp(i theta n_{p sigma}) = exp(-i t sum lam n) with t = 1, lam = -theta e_p on spin sigma
    std::vector<double> lam((size_t)N, 0.0), zero((size_t)N, 0.0);
    lam[p] = -theta;
    Program pr;
    DiagSpec d;
    d.lin_a = spin == 0 ? lam.data() : zero.data();
    d.lin_b = spin == 1 ? lam.data() : zero.data();
    pr.phase(pr.add_diag(d), -1.0);
    run_program(*plan, pr, vec, stream);
  });
}

int ffx_apply_num_num_interaction(ffx_plan plan, void* vec, double theta, int p, int sigma, int q, int tau,
                                  void* stream) {
  return guard([&] {
    if (!plan || !vec) throw Error(FFX_EINVAL, "null plan or vec");
    if (!std::isfinite(theta)) throw Error(FFX_EINVAL, "non-finite theta");
    check_orbital(*plan, p, "number-number interaction");
    check_orbital(*plan, q, "number-number interaction");
    check_spin(sigma);
    check_spin(tau);
    const int N = plan->norb;
    // phase = -(1/2 x_a^T Qa x_a + x_a^T C x_b + 1/2 x_b^T Qb x_b) must equal theta n_{p sigma} n_{q tau}
    std::vector<double> Qa((size_t)N * N, 0.0), Qb((size_t)N * N, 0.0), C((size_t)N * N, 0.0);
    if (sigma != tau) {
      if (sigma == 0)
        C[p * N + q] = -theta;
      else
        C[q * N + p] = -theta;
    } else {
      std::vector<double>& Q = sigma == 0 ? Qa : Qb;
      if (p == q) {
        Q[p * N + p] = -2.0 * theta;  // n^2 = n
      } else {
        Q[p * N + q] = -theta;
        Q[q * N + p] = -theta;
      }
    }
    Program pr;
    DiagSpec d;
    d.Qa = Qa.data();
    d.Qb = Qb.data();
    d.C = C.data();
    pr.phase(pr.add_diag(d), -1.0);
    run_program(*plan, pr, vec, stream);
  });
}

int ffx_apply_givens_rotation(ffx_plan plan, void* vec, double theta, int p, int q, int spin, void* stream) {
  return guard([&] {
    if (!plan || !vec) throw Error(FFX_EINVAL, "null plan or vec");
    if (!std::isfinite(theta)) throw Error(FFX_EINVAL, "non-finite theta");
    check_orbital(*plan, p, "Givens rotation");
    check_orbital(*plan, q, "Givens rotation");
    if (p == q) throw Error(FFX_EINVAL, "Givens rotation needs p != q");
    check_spin(spin);
    const int N = plan->norb;
    // exp(theta (E_pq - E_qp)) is the orbital rotation by expm(theta (|p><q| - |q><p|))
    std::vector<cd> U = identity(N);
    U[p * N + p] = U[q * N + q] = std::cos(theta);
    U[p * N + q] = std::sin(theta);
    U[q * N + p] = -std::sin(theta);
    rotate_one_spin(*plan, vec, U, spin, stream);
  });
}

int ffx_apply_tunneling_interaction(ffx_plan plan, void* vec, double theta, int p, int q, int spin,
                                    void* stream) {
  return guard([&] {
    if (!plan || !vec) throw Error(FFX_EINVAL, "null plan or vec");
    if (!std::isfinite(theta)) throw Error(FFX_EINVAL, "non-finite theta");
    check_orbital(*plan, p, "tunneling interaction");
    check_orbital(*plan, q, "tunneling interaction");
    if (p == q) throw Error(FFX_EINVAL, "tunneling interaction needs p != q");
    check_spin(spin);
    const int N = plan->norb;
    // exp(i theta (E_pq + E_qp)) is the orbital rotation by expm(i theta (|p><q| + |q><p|))
    std::vector<cd> U = identity(N);
    U[p * N + p] = U[q * N + q] = std::cos(theta);
    U[p * N + q] = U[q * N + p] = cd(0.0, std::sin(theta));
    rotate_one_spin(*plan, vec, U, spin, stream);
  });
}

int ffx_apply_quad_ham_evolution(ffx_plan plan, void* vec, const double* M_a, const double* M_b, double time,
                                 void* stream) {
  return guard([&] {
    if (!plan || !vec || !M_a) throw Error(FFX_EINVAL, "null plan, vec or M_a");
    const int N = plan->norb;
    if (!std::isfinite(time) || !all_finite(M_a, (size_t)2 * N * N) || (M_b && !all_finite(M_b, (size_t)2 * N * N)))
      throw Error(FFX_EINVAL, "non-finite parameter");
    // exp(-i t sum M_pq a+_p a_q) is the orbital rotation by U = expm(-i t M)
    auto to_U = [&](const double* M) {
      std::vector<cd> Mc = load_complex(N, M);
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
          if (std::abs(Mc[i * N + j] - std::conj(Mc[j * N + i])) > 1e-12 * (1.0 + std::abs(Mc[i * N + j])))
            throw Error(FFX_EINVAL, "quadratic Hamiltonian matrix is not Hermitian");
      std::vector<cd> K((size_t)N * N);
      for (int i = 0; i < N * N; ++i) K[i] = cd(0.0, -time) * Mc[i];
      return expm_antihermitian(N, K);
    };
    std::vector<cd> Ua = to_U(M_a);
    std::vector<cd> Ub = M_b ? to_U(M_b) : Ua;
    DecompPool pool;
    const Decomposition* da = pool.add(N, Ua);
    const Decomposition* db = M_b ? pool.add(N, Ub) : da;
    Program pr;
    pr.rot(da, db);
    run_program(*plan, pr, vec, stream);
  });
}

int ffx_slater_determinant(ffx_plan plan, void* vec, const int* occ_a, const int* occ_b, const double* U_a,
                           const double* U_b, void* stream) {
  return guard([&] {
    if (!plan || !vec) throw Error(FFX_EINVAL, "null plan or vec");
    ffx_plan_s& P = *plan;
    const int N = P.norb;
    // columns of U (or of the identity) in the order of the occupied orbitals
    auto minors = [&](int spin, const int* occ, const double* Um) {
      const int n = P.n[spin];
      std::vector<char> used((size_t)N, 0);
      std::vector<int> cols;
      for (int k = 0; k < n; ++k) {
        const int o = occ ? occ[k] : k;
        if (o < 0 || o >= N || used[o]) throw Error(FFX_EINVAL, "occupied orbitals must be distinct and in range");
        used[o] = 1;
      }
      // the configuration |occ> has its orbitals in ascending order
      for (int o = 0; o < N; ++o)
        if (used[o]) cols.push_back(o);
      for (int o = 0; o < N; ++o)
        if (!used[o]) cols.push_back(o);
      std::vector<cd> U = Um ? load_complex(N, Um) : identity(N);
      if (Um && unitarity_defect(N, U.data()) > 1e-10) throw Error(FFX_ENOTUNITARY, "orbital rotation is not unitary");
      std::vector<cd> V((size_t)N * N);
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) V[i * N + j] = U[i * N + cols[j]];
      return slater_column_minors(N, n, V, P.str[spin]);
    };
    if ((U_a && !all_finite(U_a, (size_t)2 * N * N)) || (U_b && !all_finite(U_b, (size_t)2 * N * N)))
      throw Error(FFX_EINVAL, "non-finite U");
    std::vector<cd> a = minors(0, occ_a, U_a);
    std::vector<cd> b = minors(1, occ_b, U_b ? U_b : U_a);
    DeviceGuard dg(P.device);
    hipStream_t s = (hipStream_t)stream;
    Upload up(&P, s);
    const double* da = up.put((const double*)a.data(), 2 * a.size());
    const double* db = up.put((const double*)b.data(), 2 * b.size());
    up.commit();
    dev::outer(P.c64, da, db, vec, P.dim[0], P.dim[1], s);
    check_launch();
  });
}

int ffx_apply_ucj(ffx_plan plan, void* vec, int n_reps, const double* U_a, const double* U_b, const double* J_aa,
                  const double* J_ab, const double* J_bb, const double* final_a, const double* final_b,
                  void* stream) {
  return guard([&] {
    if (!plan || !vec || !U_a || !J_aa) throw Error(FFX_EINVAL, "null plan, vec, U_a or J_aa");
    if (n_reps < 1) throw Error(FFX_EINVAL, "n_reps must be >= 1");
    ffx_plan_s& P = *plan;
    const int N = P.norb;
    const size_t NN = (size_t)N * N;
    const double* Jab = J_ab ? J_ab : J_aa;
    const double* Jbb = J_bb ? J_bb : J_aa;
    if (!all_finite(U_a, 2 * NN * n_reps) || (U_b && !all_finite(U_b, 2 * NN * n_reps)) ||
        !all_finite(J_aa, NN * n_reps) || !all_finite(Jab, NN * n_reps) || !all_finite(Jbb, NN * n_reps) ||
        (final_a && !all_finite(final_a, 2 * NN)) || (final_b && !all_finite(final_b, 2 * NN)))
      throw Error(FFX_EINVAL, "non-finite parameter");
    if (final_b && !final_a) throw Error(FFX_EINVAL, "final_b needs final_a");
    std::vector<std::vector<cd>> Ua, Ub;
    for (int k = 0; k < n_reps; ++k) {
      Ua.push_back(load_complex(N, U_a + 2 * NN * k));
      Ub.push_back(U_b ? load_complex(N, U_b + 2 * NN * k) : Ua.back());
      if (unitarity_defect(N, Ua.back().data()) > 1e-10 || unitarity_defect(N, Ub.back().data()) > 1e-10)
        throw Error(FFX_ENOTUNITARY, "orbital rotation is not unitary");
    }
    std::vector<cd> Fa, Fb;
    if (final_a) {
      Fa = load_complex(N, final_a);
      Fb = final_b ? load_complex(N, final_b) : Fa;
    }
    // psi = [final] prod_{k = R..1} U_k D_k U_k^dag |HF>: the Slater determinant U_1^dag|HF>, then
    // D_k and the merged rotation U_{k+1}^dag U_k (the last: final U_R, or U_R)
    auto a = slater_column_minors(N, P.n[0], dagger(N, Ua[0]), P.str[0]);
    auto b = slater_column_minors(N, P.n[1], dagger(N, Ub[0]), P.str[1]);
    DecompPool pool;
    Program pr;
    for (int k = 0; k < n_reps; ++k) {
      DiagSpec d;
      d.Qa = J_aa + NN * k;
      d.Qb = Jbb + NN * k;
      d.C = Jab + NN * k;
      pr.phase(pr.add_diag(d), -1.0);
      auto next = [&](const std::vector<std::vector<cd>>& U, const std::vector<cd>& F) {
        if (k + 1 < n_reps) return matmul(N, dagger(N, U[k + 1]), U[k]);
        return F.empty() ? U[k] : matmul(N, F, U[k]);
      };
      const Decomposition* ra = pool.add(N, next(Ua, Fa));
      const Decomposition* rb = pool.add(N, next(Ub, Fb));
      pr.rot(ra, rb);
    }
    DeviceGuard dg(P.device);
    hipStream_t s = (hipStream_t)stream;
    Upload up(&P, s);
    const double* da = up.put((const double*)a.data(), 2 * a.size());
    const double* db = up.put((const double*)b.data(), 2 * b.size());
    Compiled c = compile_program(P, up, pr, FINAL_STORE, s);
    up.commit();
    dev::outer(P.c64, da, db, vec, P.dim[0], P.dim[1], s);
    check_launch();
    execute_program(P, c, vec, vec, nullptr, s);
  });
}
