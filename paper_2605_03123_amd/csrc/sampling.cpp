// C ABI: sampling of configurations from a state vector and from a Slater
// determinant (Sec. 4.5.4, 6.1).  The host checks the inputs, moves the
// caller's uniform random numbers to the device and the results back.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "device.h"
#include "drivers.h"
#include "ffx.h"
#include "host.h"
#include "plan.h"

using namespace ffx;

namespace {

// device buffer freed at scope exit (after the stream has been synchronized)
struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t bytes) {
    if (bytes && (fault_hit("alloc") || hipMalloc(&p, bytes) != hipSuccess))
      throw Error(FFX_ENOMEM, "device allocation failed");
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

void check_uniforms(const double* u, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!(u[i] >= 0.0 && u[i] < 1.0)) throw Error(FFX_EINVAL, "uniforms must lie in [0, 1)");
}

}  // namespace

int ffx_sample_state(ffx_plan plan, const void* vec, const double* u, int64_t n_samples, int64_t* out,
                     void* stream) {
  return guard([&] {
    if (!plan || !vec || (n_samples > 0 && (!u || !out))) throw Error(FFX_EINVAL, "null pointer");
    if (n_samples < 0 || n_samples >= ((int64_t)1 << 31)) throw Error(FFX_EINVAL, "n_samples out of range");
    check_uniforms(u, n_samples);
    ffx_plan_s& P = *plan;
    DeviceGuard dg(P.device);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = P.elems();
    const int nb = dev::sample_blocks(n);
    DevBuf sums((size_t)2 * nb * 8);  // block sums and their prefix
    double* bs = (double*)sums.p;
    double* pre = bs + nb;
    // block sums, their prefix and the searches in one sequence; the total is
    // checked before any sample is handed back (the searches read only inside
    // the state and the prefix whatever the total is)
    DevBuf du((size_t)n_samples * 8), dout((size_t)n_samples * 8);
    if (n_samples > 0) HIPCHK(hipMemcpyAsync(du.p, u, (size_t)n_samples * 8, hipMemcpyHostToDevice, s));
    dev::sample_state(P.c64, vec, n, bs, pre, (const double*)du.p, n_samples, (int64_t*)dout.p, s);
    check_launch();
    double total = 0;
    HIPCHK(hipMemcpyAsync(&total, pre + nb - 1, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!(total > 0.0) || !std::isfinite(total)) throw Error(FFX_EINVAL, "state has no finite nonzero norm");
    if (n_samples == 0) return;
    HIPCHK(hipMemcpyAsync(out, dout.p, (size_t)n_samples * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  });
}

int ffx_sample_state_noalloc(ffx_plan plan, const void* vec, const double* u, int64_t n_samples, int64_t* out,
                             void* stream) {
  return guard([&] {
    if (!plan || !vec || (n_samples > 0 && (!u || !out))) throw Error(FFX_EINVAL, "null pointer");
    if (n_samples < 0 || n_samples >= ((int64_t)1 << 31)) throw Error(FFX_EINVAL, "n_samples out of range");
    ffx_plan_s& P = *plan;
    const int64_t n = P.elems();
    const int nb = dev::sample_blocks(n);
    if (nb > dev::kScratchBlocks)
      throw Error(FFX_EUNSUPPORTED, "state of " + std::to_string(n) + " amplitudes exceeds the allocation-free "
                                    "sampler's limit of " + std::to_string(dev::kScratchBlocks * 1024) + " amplitudes");
    DeviceGuard dg(P.device);
    double* scr = nullptr;
    HIPCHK(dev::sample_scratch(P.device, &scr));
    dev::sample_state(P.c64, vec, n, scr, scr + nb, u, n_samples, out, (hipStream_t)stream);
    check_launch();
  });
}

int ffx_sample_slater(ffx_plan plan, const int* occ_a, const int* occ_b, const double* U_a, const double* U_b,
                      const double* u_a, const double* u_b, int64_t n_samples, uint64_t* masks_a,
                      uint64_t* masks_b, void* stream) {
  return guard([&] {
    if (!plan) throw Error(FFX_EINVAL, "null plan");
    if (n_samples < 0 || n_samples >= ((int64_t)1 << 31)) throw Error(FFX_EINVAL, "n_samples out of range");
    ffx_plan_s& P = *plan;
    const int N = P.norb;
    if ((U_a && !all_finite(U_a, (size_t)2 * N * N)) || (U_b && !all_finite(U_b, (size_t)2 * N * N)))
      throw Error(FFX_EINVAL, "non-finite U");
    DeviceGuard dg(P.device);
    hipStream_t s = (hipStream_t)stream;
    for (int spin = 0; spin < 2; ++spin) {
      const int eta = P.n[spin];
      const int* occ = spin == 0 ? occ_a : occ_b;
      const double* Um = spin == 0 ? U_a : (U_b ? U_b : U_a);
      const double* u = spin == 0 ? u_a : u_b;
      uint64_t* masks = spin == 0 ? masks_a : masks_b;
      if (n_samples == 0) continue;
      if (!masks || (eta > 0 && !u)) throw Error(FFX_EINVAL, "null uniforms or output");
      if (eta == 0) {
        for (int64_t k = 0; k < n_samples; ++k) masks[k] = 0;
        continue;
      }
      check_uniforms(u, n_samples * eta);
      std::vector<char> used((size_t)N, 0);
      for (int k = 0; k < eta; ++k) {
        const int o = occ ? occ[k] : k;
        if (o < 0 || o >= N || used[o]) throw Error(FFX_EINVAL, "occupied orbitals must be distinct and in range");
        used[o] = 1;
      }
      std::vector<cd> U((size_t)N * N, 0.0);
      if (Um) {
        U = load_complex(N, Um);
        if (unitarity_defect(N, U.data()) > 1e-10) throw Error(FFX_ENOTUNITARY, "orbital rotation is not unitary");
      } else {
        for (int i = 0; i < N; ++i) U[i * N + i] = 1.0;
      }
      // Q = U[:, occ] with the occupied orbitals in ascending order (the distribution does not depend on it)
      std::vector<double> Q((size_t)2 * N * eta);
      for (int j = 0; j < N; ++j) {
        int c = 0;
        for (int o = 0; o < N; ++o)
          if (used[o]) {
            Q[(j * eta + c) * 2] = U[j * N + o].real();
            Q[(j * eta + c) * 2 + 1] = U[j * N + o].imag();
            ++c;
          }
      }
      DevBuf dq(Q.size() * 8), du((size_t)n_samples * eta * 8), dm((size_t)n_samples * 8);
      HIPCHK(hipMemcpyAsync(dq.p, Q.data(), Q.size() * 8, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(du.p, u, (size_t)n_samples * eta * 8, hipMemcpyHostToDevice, s));
      dev::dpp_sample((const double*)dq.p, N, eta, (const double*)du.p, n_samples, (uint64_t*)dm.p, s);
      check_launch();
      HIPCHK(hipMemcpyAsync(masks, dm.p, (size_t)n_samples * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
  });
}
