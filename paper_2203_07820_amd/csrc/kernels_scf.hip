// Elementwise kernels of the self-consistent field loop (Section 3,
// Algorithm 1): the right-hand side of the Hartree problem, the Jacobi
// preconditioner, the effective potential with LDA exchange, and the
// weighted vectors of the mixing.  All are single passes over M values.
#include <cmath>

#include "internal.h"

namespace chfsi {
namespace {

__global__ void __launch_bounds__(256)
hartree_rhs_kernel(const double* __restrict__ rho, double rho_bar, const double* __restrict__ sqm,
                   double* __restrict__ b, int64_t n) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) b[i] = 4.0 * M_PI * sqm[i] * (rho[i] - rho_bar);
}

__global__ void __launch_bounds__(256)
ediv_kernel(const double* __restrict__ x, const double* __restrict__ d, double* __restrict__ y, int64_t n) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) y[i] = x[i] / d[i];
}

__global__ void __launch_bounds__(256)
emul_kernel(const double* __restrict__ x, const double* __restrict__ d, double* __restrict__ y, int64_t n) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) y[i] = x[i] * d[i];
}

// V = V_ext + v_H - (3 rho / pi)^(1/3)
__global__ void __launch_bounds__(256)
veff_kernel(const double* __restrict__ vext, const double* __restrict__ vh, const double* __restrict__ rho,
            double* __restrict__ V, int64_t n) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) V[i] = vext[i] + vh[i] - cbrt(3.0 * fmax(rho[i], 0.0) / M_PI);
}

unsigned nblk(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

}  // namespace

hipError_t launch_hartree_rhs(const double* rho, double rho_bar, const double* sqm, double* b, int64_t n,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(hartree_rhs_kernel, dim3(nblk(n)), dim3(256), 0, s, rho, rho_bar, sqm, b, n);
  return hipGetLastError();
}

hipError_t launch_ediv(const double* x, const double* d, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ediv_kernel, dim3(nblk(n)), dim3(256), 0, s, x, d, y, n);
  return hipGetLastError();
}

hipError_t launch_emul(const double* x, const double* d, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(emul_kernel, dim3(nblk(n)), dim3(256), 0, s, x, d, y, n);
  return hipGetLastError();
}

hipError_t launch_veff(const double* vext, const double* vh, const double* rho, double* V, int64_t n,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(veff_kernel, dim3(nblk(n)), dim3(256), 0, s, vext, vh, rho, V, n);
  return hipGetLastError();
}

}  // namespace chfsi
