// Loss head of the flow-control forcing (Sec. 3.2): the shell energy spectrum of a
// velocity field's Fourier coefficients, the gradient of the log-spectrum cost applied
// to those coefficients, and the scaled real part of the inverse transform (the
// velocity shift of the controlled step).  The transforms themselves are the caller's.
//
// With uh_a(k) the unnormalised forward transform of u_a and s = 1/N:
//   E(K) = s^2/2 * sum_{k in shell K} sum_a |uh_a(k)|^2,
//   R    = sum_{K = k_lo..k_hi} (ln max(E_K, c) - ln max(Et_K, c))^2,
//   dR/du_a(x) = Re IFFT_norm(g * s * uh_a)(x) with g(k) = dR/dE at the shell of k,
// since E is a sum of squared moduli of linear functions of u.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"

namespace lbm {
namespace {

// One block per shell K; thread t takes the shell's members t, t + 256, ... in order,
// then a fixed tree over the threads, so every call sums alike.  Offsets and indices
// outside the table are clamped or skipped (an invalid table gives wrong sums, never an
// access outside uh).
__global__ __launch_bounds__(256) void shell_energy_kernel(const double2* __restrict__ uh, int D, uint32_t n,
                                                           const int32_t* __restrict__ order,
                                                           const int32_t* __restrict__ offsets, double half_s2,
                                                           double* __restrict__ E) {
  const int K = blockIdx.x;
  const int32_t b = min(max(offsets[K], 0), (int32_t)n);
  const int32_t e = min(max(offsets[K + 1], b), (int32_t)n);
  double acc = 0;
  for (int32_t i = b + (int32_t)threadIdx.x; i < e; i += 256) {
    const uint32_t k = (uint32_t)order[i];
    if (k >= n) continue;
    for (int a = 0; a < D; ++a) {
      const double2 z = uh[(uint64_t)a * n + k];
      acc += z.x * z.x + z.y * z.y;
    }
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) E[K] = half_s2 * sh[0];
}

// uh_a(k) *= scale * dR/dE_K at the shell K of k: 2 (ln E_K - ln max(Et_K, c)) / E_K
// inside the band where E_K >= c, zero elsewhere (the clamp at c is flat below it).
// If R is given, block 0 also writes the cost: thread t sums the band's shells t,
// t + 256, ... in order, then a fixed tree over the threads.
__global__ __launch_bounds__(256) void log_spectrum_grad_kernel(double2* __restrict__ uh, int D, uint32_t n,
                                                                const int32_t* __restrict__ shell,
                                                                const double* __restrict__ E,
                                                                const double* __restrict__ Et, int nshell, int k_lo,
                                                                int k_hi, double c, double scale,
                                                                double* __restrict__ R) {
  const uint64_t k = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (R && blockIdx.x == 0) {  // uniform over the block: every thread reaches the barriers
    double r = 0;
    for (int K = k_lo + (int)threadIdx.x; K <= k_hi; K += 256) {
      const double d = log(fmax(E[K], c)) - log(fmax(Et[K], c));
      r += d * d;
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) *R = sh[0];
  }
  if (k >= n) return;
  const int K = shell[k];
  double g = 0;
  if (K >= k_lo && K <= k_hi && K < nshell) {
    const double EK = E[K];
    if (EK >= c) g = 2.0 * (log(EK) - log(fmax(Et[K], c))) / EK * scale;
  }
  for (int a = 0; a < D; ++a) {
    double2 z = uh[(uint64_t)a * n + k];
    z.x *= g;
    z.y *= g;
    uh[(uint64_t)a * n + k] = z;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void real_part_kernel(const double2* __restrict__ z, uint64_t count, double scale,
                                                        T* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i < count) out[i] = static_cast<T>(scale * z[i].x);
}

unsigned blocks_for(uint64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

hipError_t launch_shell_energy(const void* uh, int D, uint32_t n, const int32_t* order, const int32_t* offsets,
                               int nshell, double scale, double* E, hipStream_t s) {
  shell_energy_kernel<<<(unsigned)nshell, 256, 0, s>>>((const double2*)uh, D, n, order, offsets,
                                                        0.5 * scale * scale, E);
  return hipGetLastError();
}

hipError_t launch_log_spectrum_grad(void* uh, int D, uint32_t n, const int32_t* shell, const double* E,
                                    const double* Et, int nshell, int k_lo, int k_hi, double cutoff, double scale,
                                    double* R, hipStream_t s) {
  log_spectrum_grad_kernel<<<blocks_for(n), 256, 0, s>>>((double2*)uh, D, n, shell, E, Et, nshell, k_lo, k_hi,
                                                         cutoff, scale, R);
  return hipGetLastError();
}

hipError_t launch_real_part(const void* z, uint64_t count, double scale, void* out, bool f64, hipStream_t s) {
  if (f64)
    real_part_kernel<double><<<blocks_for(count), 256, 0, s>>>((const double2*)z, count, scale, (double*)out);
  else
    real_part_kernel<float><<<blocks_for(count), 256, 0, s>>>((const double2*)z, count, scale, (float*)out);
  return hipGetLastError();
}

}  // namespace lbm
