/*
 * ffx.h - C ABI of libffx: evolution of a fermionic state vector at fixed
 * particle number and S_z on AMD MI355X (gfx950).
 *
 * The state of a sector (N_alpha, N_beta) with N spatial orbitals is the
 * dim_a x dim_b complex matrix Gamma[i_a][i_b] = gamma(I_alpha, I_beta)
 * (paper Sec. 3.1), dim_sigma = C(N, N_sigma), stored alpha-major
 * (element (i_a, i_b) at offset i_a * dim_b + i_b) as interleaved
 * (re, im) pairs: complex128 (FFX_C128) or complex64 (FFX_C64).
 * Configurations of one spin are N-bit masks (bit p set <=> orbital p
 * occupied, Sec. 2.2); address = rank in ascending integer order, so the
 * Hartree-Fock configuration {0..n-1} has address 0.
 *
 * Conventions shared by every call:
 *   - Return value: FFX_OK (0) or a negative error code.  No call aborts the
 *     process.  ffx_last_error() returns a thread-local message for the most
 *     recent failure on the calling thread.
 *   - Device pointers (vec, workspace) are caller-owned device memory on the
 *     plan's device.  Small matrices and vectors are caller-owned HOST arrays
 *     of double, read during the call only: real matrices row-major
 *     norb x norb; complex matrices row-major with interleaved (re, im).
 *   - `stream` is a hipStream_t (NULL = the default stream).  apply_* calls
 *     only enqueue work and return; energy / gradient calls synchronize the
 *     stream before returning host results.  A plan must not be used from two
 *     streams or two threads at the same time.
 *   - Orbital rotations, diagonal Coulomb and number-operator gates are applied
 *     IN PLACE to vec.
 */
#ifndef FFX_H
#define FFX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FFX_OK = 0,
  FFX_EINVAL = -1,       /* bad norb / nelec / pointer / dtype / size / parameter */
  FFX_ENOTUNITARY = -2,  /* ||U^dag U - I||_max > 1e-10 */
  FFX_ENOMEM = -3,       /* device or pinned host allocation failed */
  FFX_EDEVICE = -4,      /* a HIP runtime call failed */
  FFX_EUNSUPPORTED = -5  /* valid request this build does not implement */
};

typedef enum { FFX_C128 = 0, FFX_C64 = 1 } ffx_dtype;

typedef struct ffx_plan_s* ffx_plan;

/* Message for the last failure on this thread ("" if none). */
const char* ffx_last_error(void);

/* C(norb, n): the number of configurations of one spin (Sec. 2.6).
   Returns -1 for norb outside [1, 32] or n outside [0, norb]. */
int64_t ffx_dim(int norb, int n);

/* Host-only: the dim configurations of n electrons in norb orbitals as bit
   masks in address order (Sec. 2.2, 3.1).  out_masks holds ffx_dim(norb, n)
   entries.  Needs no GPU. */
int ffx_strings(int norb, int n, uint64_t* out_masks);

/* Host-only: decomposition of a norb x norb unitary U into adjacent Givens
   rotations and a final phase layer (Sec. 3.2.3):
     U = diag(exp(i phase)) G_K ... G_1,  K = norb (norb - 1) / 2,
   where G_k acts on orbitals (p_k, p_k + 1) as the 2x2 block
   [[c_k, s_k], [-conj(s_k), c_k]] (c_k real).  G_1 is applied to the state
   first.  Outputs: p (K ints), c (K doubles), s (K complex, interleaved),
   phase (norb doubles).  Returns FFX_ENOTUNITARY for a non-unitary U.  Needs
   no GPU. */
int ffx_givens_decomposition(int norb, const double* U, int* p, double* c, double* s,
                             double* phase);

/* A plan owns the device string tables, window tables and a small parameter
   upload ring for one (norb, n_alpha, n_beta, dtype, device).
   1 <= norb <= 32; the state must fit in device memory. */
int ffx_plan_create(ffx_plan* out, int norb, int n_alpha, int n_beta, ffx_dtype dtype,
                    int device);
int ffx_plan_destroy(ffx_plan plan);
/* dim_a, dim_b and the state size in bytes. */
int ffx_plan_info(ffx_plan plan, int64_t* dim_a, int64_t* dim_b, int64_t* state_bytes);
/* Copy of the device string table of one spin (0 = alpha, 1 = beta) to host,
   dim entries; bit-exact with ffx_strings. */
int ffx_plan_strings(ffx_plan plan, int spin, uint64_t* out_masks);

/* Orbital rotation script-U(U) = exp(sum_pq log(U)_pq a^dag_p a_q), per spin
   (Table 1, Sec. 2.3, 3.2.3).  U_a, U_b: complex norb x norb unitaries;
   U_b = NULL means U_b = U_a.  Implemented as Givens sweeps over
   configuration pairs, several rotations per pass over HBM. */
int ffx_apply_orbital_rotation(ffx_plan plan, void* vec, const double* U_a, const double* U_b,
                               void* stream);

/* The same orbital rotation in its dense form (Sec. 2.3: script-U(U) acts on
   the sector as the compound matrices, Gamma' = C_{n_a}(U_a) Gamma
   C_{n_b}(U_b)^T with C_n(U)[J, I] = det U[J, I] over ascending occupied
   orbitals): the compound matrices are built on the device, then two complex
   products run on the FP64 matrix cores.  It costs 16 d^3 flops against the
   Givens sweeps' 20 n (N - n) d^2 and exists to be measured against them on
   small sectors.  complex128 plans with at most 8 electrons and 4096
   configurations per spin (FFX_EUNSUPPORTED otherwise).  workspace: device
   buffer of ffx_workspace_bytes(plan, 3) bytes (the two compound matrices and
   one intermediate state).  Enqueues only; FFX_ENOTUNITARY as above. */
int ffx_apply_orbital_rotation_dense(ffx_plan plan, void* vec, const double* U_a, const double* U_b,
                                     void* workspace, void* stream);

/* Number-operator-sum evolution exp(-i t sum_{p,sigma} lam^sigma_p n_{p sigma})
   (Table 1, Sec. 3.2.1).  lam_a, lam_b: norb real; lam_b = NULL means lam_a.
   basis_U (complex norb x norb, NULL = none): the number operators of the
   rotated orbitals instead, script-U(B) [evolution] script-U(B)^dag. */
int ffx_apply_num_op_sum_evolution(ffx_plan plan, void* vec, const double* lam_a,
                                   const double* lam_b, double time, const double* basis_U, void* stream);

/* Diagonal Coulomb evolution
   exp(-(1/2) i t sum_{pq, sigma tau} J^{sigma tau}_pq n_{p sigma} n_{q tau})
   (Table 1, Sec. 3.2.2).  J_aa, J_bb: real symmetric norb x norb; J_ab: real
   norb x norb, J^{ba} = (J^{ab})^T; J_ab or J_bb = NULL means J_aa.  basis_U as for the
   number-operator-sum evolution (the rotated basis of Sec. 4.5.3's terms). */
int ffx_apply_diag_coulomb_evolution(ffx_plan plan, void* vec, const double* J_aa,
                                     const double* J_ab, const double* J_bb, double time,
                                     const double* basis_U, void* stream);

/* The remaining gates of Table 1, applied IN PLACE.  spin: 0 = alpha,
   1 = beta; orbital indices in [0, norb).  FFX_EINVAL for a non-finite angle,
   an index out of range or p == q where two orbitals are needed.
   Number interaction exp(i theta n_{p,spin}) (a number-operator-sum
   evolution with one nonzero coefficient). */
int ffx_apply_num_interaction(ffx_plan plan, void* vec, double theta, int p, int spin, void* stream);

/* Number-number interaction exp(i theta n_{p,sigma} n_{q,tau}) (a diagonal
   Coulomb evolution with one nonzero coupling; p == q with sigma == tau is
   exp(i theta n_{p,sigma})). */
int ffx_apply_num_num_interaction(ffx_plan plan, void* vec, double theta, int p, int sigma, int q, int tau,
                                  void* stream);

/* Givens rotation exp(theta (a^dag_{p,spin} a_{q,spin} - a^dag_{q,spin} a_{p,spin})):
   the orbital rotation of that spin by the identity with the (p, q) block
   [[cos theta, sin theta], [-sin theta, cos theta]] (Sec. 2.3); p, q need
   not be adjacent. */
int ffx_apply_givens_rotation(ffx_plan plan, void* vec, double theta, int p, int q, int spin, void* stream);

/* Tunneling interaction exp(i theta (a^dag_{p,spin} a_{q,spin} + h.c.)): the
   orbital rotation of that spin with the (p, q) block
   [[cos theta, i sin theta], [i sin theta, cos theta]]. */
int ffx_apply_tunneling_interaction(ffx_plan plan, void* vec, double theta, int p, int q, int spin,
                                    void* stream);

/* Quadratic Hamiltonian evolution exp(-i t sum_{pq,sigma} M^sigma_pq a^dag_{p sigma} a_{q sigma}):
   the orbital rotation by U = expm(-i t M) per spin.  M_a, M_b: complex
   Hermitian norb x norb (interleaved); M_b = NULL means M_a.  FFX_EINVAL for
   a matrix that is not Hermitian to 1e-12. */
int ffx_apply_quad_ham_evolution(ffx_plan plan, void* vec, const double* M_a, const double* M_b, double time,
                                 void* stream);

/* Slater determinant (Sec. 2.4): vec is OVERWRITTEN with script-U(U) |occ>,
   amplitude det U_a[I_alpha, occ_a] * det U_b[I_beta, occ_beta] with the occupied
   orbitals in ascending order.  occ_a / occ_b: n_alpha / n_beta distinct
   orbital indices in any order (NULL: the lowest orbitals, Hartree-Fock);
   U_a / U_b: complex norb x norb unitaries (NULL: the identity; U_b = NULL
   with U_a given means U_a). */
int ffx_slater_determinant(ffx_plan plan, void* vec, const int* occ_a, const int* occ_b, const double* U_a,
                           const double* U_b, void* stream);

/* Unitary cluster Jastrow ansatz with per-spin rotations and full
   diagonal-Coulomb matrices (Sec. 4.5.1; the LUCJ entry point below is its
   restricted, parameterized form): vec is OVERWRITTEN with
   [script-U(F)] prod_{k = n_reps..1} [script-U(U_k) D_k script-U(U_k)^dag] |HF>,
   D_k = the diagonal Coulomb evolution at t = 1 with (J_aa[k], J_ab[k], J_bb[k]).
   U_a, U_b: n_reps complex norb x norb unitaries each (U_b = NULL: U_a);
   J_aa, J_ab, J_bb: n_reps real norb x norb (J_ab or J_bb = NULL: J_aa);
   final_a, final_b: the optional final rotation F per spin (NULL: none;
   final_b = NULL with final_a given means final_a). */
int ffx_apply_ucj(ffx_plan plan, void* vec, int n_reps, const double* U_a, const double* U_b, const double* J_aa,
                  const double* J_ab, const double* J_bb, const double* final_a, const double* final_b,
                  void* stream);

/* Sampling of configurations from the state (Sec. 6.1, sample-based
   algorithms): for each uniform u[k] in [0, 1) (host, n_samples of them),
   out[k] (host int64) is the address i_a * dim_b + i_b of the first
   configuration, in address order, whose cumulative probability
   sum |gamma|^2 exceeds u[k] times the total (accumulated in FP64 in a fixed
   order; zero-probability configurations are never returned).  vec is read
   only and need not be normalised.  Synchronizes.  FFX_EINVAL for a uniform
   outside [0, 1) or a state with no finite nonzero norm. */
int ffx_sample_state(ffx_plan plan, const void* vec, const double* u, int64_t n_samples, int64_t* out,
                     void* stream);

/* Allocation-free variant of ffx_sample_state, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc): it calls no allocating routine and only
   enqueues work on `stream`.  u (n_samples uniforms) and out (n_samples
   int64) are DEVICE buffers on the plan's device; out[k] is the address
   ffx_sample_state returns for u[k], or -1 for a uniform outside [0, 1) or a
   state with no finite nonzero norm (checked on the device, not reported
   through the return code).  The block sums of |gamma|^2 and their prefix go
   to a static device array of the library (4 MiB per device, held until the
   process ends), so states of at most 2^28 amplitudes are accepted
   (FFX_EUNSUPPORTED above that).  Every call on one device shares that
   array: calls that overlap on one device (two streams, two threads) race,
   and each call overwrites what the last one left there. */
int ffx_sample_state_noalloc(ffx_plan plan, const void* vec, const double* u, int64_t n_samples, int64_t* out,
                             void* stream);

/* Sampling of configurations from the Slater determinant script-U(U)|occ>
   (Sec. 4.5.4) without forming the state: per spin an independent draw from
   p(I) = |det U[I, occ]|^2, one orbital at a time from its conditional
   distribution given the orbitals drawn so far (the projection
   determinantal point process with kernel U[:, occ] U[:, occ]^dag;
   O(n^2 norb) per sample).  Step k of sample s uses u_sigma[s * n_sigma + k]
   (host, uniforms in [0, 1)): the first orbital, in orbital order, whose
   cumulative conditional weight exceeds u times the total.  occ_a / occ_b:
   occupied orbitals (NULL: the lowest); U_a / U_b: complex norb x norb
   unitaries (NULL: the identity; U_b = NULL with U_a given means U_a).
   masks_a / masks_b (host, n_samples each): the sampled configurations as
   bit masks.  Synchronizes. */
int ffx_sample_slater(ffx_plan plan, const int* occ_a, const int* occ_b, const double* U_a, const double* U_b,
                      const double* u_a, const double* u_b, int64_t n_samples, uint64_t* masks_a,
                      uint64_t* masks_b, void* stream);

/* Double-factorized Hamiltonian (Eq. double-factorized-hamiltonian):
   H = sum h_pq a^dag_{p s} a_{q s} + 1/2 sum_t sum J^(t)_pq n^(t)_{p s} n^(t)_{q t'}.
   h: real symmetric norb^2; J: n_terms * norb^2 real symmetric;
   U: n_terms * norb^2 complex unitaries (interleaved). */
typedef struct {
  int norb;
  int n_terms;
  const double* h;
  const double* J;
  const double* U;
} ffx_df_ham;

/* Trotter-Suzuki evolution exp(-i H T) ~ S_order(T / n_steps)^n_steps with
   T = dt * n_steps (Sec. 4.5.3).  order 0: S_0 (one-body term first, then the
   two-body terms in array order); order 1: the symmetric S_1; order k >= 2:
   Suzuki's recursion.  Adjacent orbital rotations are merged through
   script-U(U) script-U(V) = script-U(UV) (Sec. 2.3). */
int ffx_apply_df_trotter_step(ffx_plan plan, void* vec, const ffx_df_ham* ham, double dt,
                              int n_steps, int order, void* stream);

/* Trotter-Suzuki evolution under a diagonal Coulomb Hamiltonian
   (Eq. diagonal-coulomb-hamiltonian, Sec. 4.5.3):
     H = sum_{pq,sigma} h_pq a^dag_{p sigma} a_{q sigma}
       + 1/2 sum_{pq,sigma tau} J^{sigma tau}_pq n_{p sigma} n_{q tau},
   as the sum of two terms, H_1 = the one-body term (applied first) and H_2 =
   the diagonal Coulomb term, each evolved exactly: exp(-i t H_1) is the
   orbital rotation by exp(-i t h) on both spins (Table 1, quadratic
   Hamiltonian evolution), exp(-i t H_2) the diagonal Coulomb evolution.
   vec <- S_order(dt)^n_steps vec, with order 0 (S_0), 1 (S_1) or k >= 2
   (Suzuki's S_k) as in ffx_apply_df_trotter_step.  h: real symmetric
   norb x norb (FFX_EINVAL if not symmetric to 1e-12); J_aa, J_bb: real
   symmetric; J_ab: real, J^{beta alpha} = (J_ab)^T; J_ab or J_bb = NULL means
   J_aa.  Enqueues only. */
int ffx_simulate_trotter_diag_coulomb(ffx_plan plan, void* vec, const double* h, const double* J_aa,
                                      const double* J_ab, const double* J_bb, double dt, int n_steps, int order,
                                      void* stream);

/* LUCJ ansatz (Sec. 4.5.1): vec is OVERWRITTEN with
   prod_{k = n_reps..1} [script-U(U_k) D_k script-U(U_k)^dag] |HF>.
   Per repetition the flat real parameter block is
   [Re A (norb^2), Im A (norb^2), j_same (norb - 1), j_opp (norb)],
   U_k = expm(A - A^dag) for both spins, D_k = diagonal Coulomb evolution at
   t = 1 with J^{aa} = J^{bb} holding j_same[p] at (p, p+1) and (p+1, p),
   J^{ab} = diag(j_opp).  n_params = n_reps (2 norb^2 + 2 norb - 1). */
typedef struct {
  int norb;
  int n_reps;
  const double* params;
} ffx_lucj;

int ffx_lucj_n_params(int norb, int n_reps);
int ffx_apply_lucj(ffx_plan plan, void* vec, const ffx_lucj* op, void* stream);

/* Workspace size in bytes: what = 0 for ffx_df_energy and
   ffx_apply_df_hamiltonian (one state), 1 for the gradients, 2 for
   ffx_df_evolve_exact (four states), 3 for ffx_apply_orbital_rotation_dense. */
int64_t ffx_workspace_bytes(ffx_plan plan, int what);

/* Energy <psi|H|psi> of vec for the DF Hamiltonian (Sec. 4.2), evaluated as
   sum_t sum_I w_t(I) |(script-U(U_t)^dag psi)(I)|^2 with the one-body term in
   the eigenbasis of h; FP64 accumulation in a fixed order, so repeated calls
   give identical results.  workspace: device buffer of
   ffx_workspace_bytes(plan, 0) bytes.  Synchronizes the stream. */
int ffx_df_energy(ffx_plan plan, const void* vec, const ffx_df_ham* ham, double* energy,
                  void* workspace, void* stream);

/* Action of the DF Hamiltonian (Eq. double-factorized-hamiltonian, in the
   form of Sec. 4.2): out = H vec = sum_t script-U(W_t) D_t script-U(W_t)^dag vec
   with W_0 the eigenvectors of h and D_0 = sum_p eps_p N_p, W_t = U_t and
   D_t = 1/2 sum_pq J_t[p][q] N_p N_q (N_p = n_{p alpha} + n_{p beta}).  vec
   (read only), out and workspace (ffx_workspace_bytes(plan, 0) bytes) are
   distinct device buffers; FFX_EINVAL when two of them are the same pointer.
   The one-body term is applied either through the eigenbasis of h (two
   orbital rotations) or, when its excitation tables are short (sparse h or few
   electrons: at most 48 entries per configuration over both spins), directly
   as sum_pq h_pq E_pq from those tables; the environment variable
   FFX_ONEBODY=rot|direct forces one route.  The direct route allocates its
   tables for the call and waits for the device before returning; otherwise
   the call only enqueues. */
int ffx_apply_df_hamiltonian(ffx_plan plan, const void* vec, void* out, const ffx_df_ham* ham, void* workspace,
                             void* stream);

/* Exact time evolution vec <- exp(-i H time) vec for the DF Hamiltonian, the
   reference that Trotter errors are measured against (Sec. 6.2, estimating
   Trotter error), by a Chebyshev expansion of the exponential in the
   Hamiltonian action above.  The spectrum of H in the plan's sector is
   enclosed in [lo, hi] from the terms' weights (one-body term: the sums of the
   n lowest and n highest eigenvalues of h per spin; term t: the eigenvalue
   range of J_t times the range of |x|^2 over occupation vectors x); with
   c = (lo + hi) / 2 and r = (hi - lo) / 2,
     exp(-i H time) = exp(-i c time) sum_k (2 - delta_k0) (-i)^k J_k(r time) T_k((H - c) / r)
   (J_k Bessel functions of the first kind, T_k Chebyshev polynomials).  The
   series stops at the first K whose dropped terms weigh at most tol / 2 in
   total (2 sum_{k > K} |J_k(r |time|)|), so the truncation error is below
   tol / 2 times ||vec|| in exact arithmetic; rounding adds about K times the
   unit roundoff of the state's type (complex64: tol below about 1e-5 is not
   reached).  n_matvec (host, may be NULL) receives K, the number of
   Hamiltonian actions.  workspace: ffx_workspace_bytes(plan, 2) bytes, not
   overlapping vec.  Enqueues only.  FFX_EINVAL for a non-finite time or a tol
   that is not positive; FFX_EUNSUPPORTED when r |time| exceeds about 1e6. */
int ffx_df_evolve_exact(ffx_plan plan, void* vec, const ffx_df_ham* ham, double time, double tol, void* workspace,
                        int* n_matvec, void* stream);

/* Euclidean distance ||x - y||_2 of two states of the plan (device, read
   only), accumulated in FP64 in a fixed order: the Trotter error measure of
   Sec. 6.2.  Synchronizes the stream. */
int ffx_state_distance(ffx_plan plan, const void* x, const void* y, double* dist, void* stream);

/* LUCJ energy E(theta) = <psi(theta)|H|psi(theta)> and its gradient
   dE/dtheta (n_params doubles) by the adjoint method: the costate
   lambda = H psi is pulled back through the gates while psi is uncomputed,
   so no intermediate state is stored.  workspace: ffx_workspace_bytes(plan, 1)
   bytes.  psi_out (device, may be NULL) receives psi(theta).  Synchronizes. */
int ffx_lucj_energy_grad(ffx_plan plan, const ffx_lucj* op, const ffx_df_ham* ham,
                         double* energy, double* grad, void* psi_out, void* workspace,
                         void* stream);

/* Energy after a DF Trotter chain and its gradient by the adjoint method:
   E = Re <psi_T|H_obs|psi_T>, psi_T = S_0(dt)^n_steps psi_0 (Sec. 4.5.3, one-body
   term first) under the evolution Hamiltonian `ham` = (h, J_t, U_t), with the
   observable `obs` held fixed (the paper does not define this gradient; this
   is the library's extension).  The costate lambda = H_obs psi_T is pulled
   back through every gate while psi is uncomputed; no intermediate state is
   stored.  vec0 (device, read only): psi_0.  Outputs (host):
     grad_h[p*N+q]      dE for moving h_pq and h_qp together (one entry when p == q)
     grad_J[t*N*N+p*N+q] the same for J_t
     grad_U[t*2N^2 + k]  U_t -> U_t expm(A - A^dag) at A = 0: k < N^2 is d/d Re A_pq,
                         k >= N^2 is d/d Im A_pq (the LUCJ layout)
   grad_J / grad_U may be NULL only when ham->n_terms == 0.  workspace:
   ffx_workspace_bytes(plan, 1) bytes; psi_out (device, may be NULL) receives
   psi_T.  Synchronizes the stream.  The plan's device result block grows to
   9 N^2 n_terms + 4 N^2 doubles when needed (that first call waits for the
   device before replacing it). */
int ffx_df_chain_energy_grad(ffx_plan plan, const void* vec0, const ffx_df_ham* ham, const ffx_df_ham* obs,
                             double dt, int n_steps, double* energy, double* grad_h, double* grad_J,
                             double* grad_U, void* psi_out, void* workspace, void* stream);

/* ---------------------------------------------------------------------------
   Batched LUCJ energy + adjoint gradient over many independent sectors of
   uneven size (each instance its own norb, (n_alpha, n_beta), LUCJ
   parameters and DF Hamiltonian), all of them together: one kernel launch
   per pass level, shared by every instance (Sec. 4.5.1 ansatz, Sec. 4.2
   energy; the batching itself is this library's extension).
   A batch object owns one plan per distinct sector type and the class tables
   of the batched kernel.  Limits: 8 <= norb <= 16 for complex64 and
   6 <= norb <= 16 for complex128, and one row of every sector must fit in LDS
   (norb <= 16 at half filling); otherwise FFX_EUNSUPPORTED.
   --------------------------------------------------------------------------- */
typedef struct ffx_batch_s* ffx_batch;

int ffx_batch_create(ffx_batch* out, int n_inst, const int* norb, const int* n_alpha,
                     const int* n_beta, ffx_dtype dtype, int device);
int ffx_batch_destroy(ffx_batch batch);

/* Device workspace for ffx_batch_lucj_energy_grad: three states per instance
   (psi, lambda, a temporary), each rounded up to 256 bytes. */
int64_t ffx_batch_workspace_bytes(ffx_batch batch);

/* ops[i], hams[i]: the instance's LUCJ operator and DF Hamiltonian (host data,
   read during the call).  energies: n_inst doubles; grads: the instances'
   gradients back to back (ffx_lucj_n_params(norb_i, n_reps_i) each, in
   instance order).  Runs every instance's forward pass, costate, energy and
   reverse sweep on `stream`, then synchronizes: the passes of all instances
   are grouped by level (pass k of every instance), and each level runs as one
   kernel launch per pass kind, one block per task (a block of rows or columns
   of one instance's state); with ffx_batch_single_launch(batch, 1), the whole
   batch is ONE cooperative launch whose blocks take each level's tasks with a
   grid barrier between levels.  A persistent launch over a task queue with
   per-instance dependency counters is built but switched off
   (ffx_batch_persistent). */
int ffx_batch_lucj_energy_grad(ffx_batch batch, const ffx_lucj* ops, const ffx_df_ham* hams,
                               double* energies, double* grads, void* workspace, void* stream);

/* Autotuner: times ffx_batch_lucj_energy_grad on the given instances for each
   candidate (rows of a task, through the target number of elements a task
   holds in LDS, x the largest number of Givens rotations fused into one
   stage) and keeps the fastest for later calls.  Writes the chosen target
   elements and stage depth to *target_elems and *stage_rots (may be NULL). */
int ffx_batch_tune(ffx_batch batch, const ffx_lucj* ops, const ffx_df_ham* hams, void* workspace,
                   void* stream, int* target_elems, int* stage_rots);

/* enable != 0: calls run the whole batch as ONE cooperative launch
   (hipLaunchCooperativeKernel) whose blocks walk the pass levels in order,
   taking each level's tasks from a counter, with a grid barrier between
   levels; its results equal those of the per-level launches (the same tasks
   in the same arithmetic order).  The grid is the number of blocks that fit
   the device at once (none fitting: per-level launches); FFX_EDEVICE if the
   cooperative launch is refused.  enable = 0 (the default): one launch per
   pass kind of each level, each with only its kind's code and LDS, so more
   blocks share a compute unit. */
int ffx_batch_single_launch(ffx_batch batch, int enable);

/* Timing of the last ffx_batch_lucj_energy_grad: device time from the first to
   the last launch (HIP events on the call's stream), wall time of the whole
   call (host preparation, launches, result copy, gradient chain rules) and the
   number of kernel launches. */
int ffx_batch_timing(ffx_batch batch, double* device_ms, double* call_ms, int* launches);

/* Configuration in use (for reports): target elements per task, stage depth,
   resident blocks of a launch that holds the whole device (the task-queue
   launch; the cooperative launch sizes its grid the same way for its own
   kernel), and the LDS bytes per block. */
int ffx_batch_info(ffx_batch batch, int* target_elems, int* stage_rots, int* blocks, int64_t* lds_bytes);

/* Diagnostics of the batched task queue: builds every instance's passes for
   these operators and Hamiltonians exactly as ffx_batch_lucj_energy_grad does
   (programs compiled, tables uploaded on `stream`), launches none of them, and
   writes the queue in task order, one row of six int64 per pass: pass level,
   instance, pass kind, tasks, dependency count (tasks of the instance's
   earlier passes that must have finished before any task of this pass
   starts) and the pass's first task in the queue.  *n_passes: the number of
   rows; table may be NULL to ask for it; cap (rows) < *n_passes gives
   FFX_EINVAL. */
int ffx_batch_queue(ffx_batch batch, const ffx_lucj* ops, const ffx_df_ham* hams, void* workspace, void* stream,
                    int64_t* table, int64_t cap, int64_t* n_passes);

/* The persistent launch over that queue (blocks take tasks from one atomic
   counter and wait on per-instance counters of finished tasks).  Switched off:
   enable != 0 gives FFX_EUNSUPPORTED, enable = 0 succeeds. */
int ffx_batch_persistent(ffx_batch batch, int enable);

/* Diagnostics: per-launch timing of the dominant kernels.  While enabled,
   each segment pass and each window pass is bracketed by HIP events on the
   stream it is launched on.  ffx_timing_enable resets the counters
   (enable = 0 stops recording).  ffx_timing_read synchronizes on the recorded
   events and returns, for `which` = 2 * kind + spin (kind 0 = window passes,
   1 = segment passes, 2 = segment passes on row planes; spin = the spin whose configurations the launch
   rotates): the summed kernel time in ms, the number of launches, the
   algorithmic bytes those launches stand for (a launch applying r of the
   K = norb (norb - 1) / 2 rotations of one spin counts r / K of one read plus
   one write of the state) and their algorithmic VALU slots (per rotated
   configuration pair: 8 for a real rotation, 12 for a complex one). */
int ffx_timing_enable(ffx_plan plan, int enable);
int ffx_timing_read(ffx_plan plan, int which, double* total_ms, int64_t* launches,
                    double* algorithmic_bytes, double* valu_slots);

#ifdef __cplusplus
}
#endif

#endif /* FFX_H */
