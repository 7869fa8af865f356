// Kernels of the self-consistent field loop (Section 3, Algorithm 1): the
// stiffness operator of the Hartree problem applied to one vector by sum
// factorisation, and single passes over M values for its right-hand side,
// the Jacobi preconditioner, the effective potential with LDA exchange and
// the weighted vectors of the mixing.
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

struct StiffArgs {
  const double* u;       // M values
  const double* dscale;  // M^-1/2 per node
  double* q;             // M values, accumulated
  int nc, n;             // cells and nodes per side
  double K1[64];         // 1D stiffness, row-major (p+1) x (p+1)
  double M1[64];         // 1D consistent mass
};

// One line of a 1D operator along stride `st`: out[i] = sum_j T[i][j] in[j].
template <int Q>
__device__ __forceinline__ void line_apply(const double* T, const double* in, double* out, int base, int st) {
  double v[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) v[j] = in[base + st * j];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    double o = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j) o = fma(T[i * Q + j], v[j], o);
    out[base + st * i] = o;
  }
}

// q += D K D u for one cell per workgroup (one wave): the cell stiffness
// K^c = M1 (x) M1 (x) K1 + M1 (x) K1 (x) M1 + K1 (x) M1 (x) M1 applied by sum
// factorisation, y = M1_z (M1_y K1_x x + K1_y M1_x x) + K1_z M1_y M1_x x,
// seven passes of a (p+1) x (p+1) matrix over the cell's lines in LDS.
template <int P>
__global__ void __launch_bounds__(64) stiffness_kernel(StiffArgs a) {
  constexpr int Q = P + 1, MC = Q * Q * Q, L = Q * Q;
  __shared__ double x[MC], ux[MC], vx[MC], s1[MC], s2[MC];
  __shared__ int32_t node[MC];
  const int t = threadIdx.x;
  const int64_t e = blockIdx.x;
  const int cx = static_cast<int>(e % a.nc), cy = static_cast<int>((e / a.nc) % a.nc),
            cz = static_cast<int>(e / (static_cast<int64_t>(a.nc) * a.nc));
  for (int l = t; l < MC; l += 64) {
    const int ax = l % Q, ay = (l / Q) % Q, az = l / L;
    const int nd = (cx * P + ax) % a.n + a.n * ((cy * P + ay) % a.n + a.n * ((cz * P + az) % a.n));
    node[l] = nd;
    x[l] = a.dscale[nd] * a.u[nd];
  }
  __syncthreads();
  // x direction (lines along a: base = Q (b + Q c), stride 1)
  for (int li = t; li < L; li += 64) {
    line_apply<Q>(a.K1, x, ux, li * Q, 1);
    line_apply<Q>(a.M1, x, vx, li * Q, 1);
  }
  __syncthreads();
  // y direction (base = a + Q^2 c, stride Q): s1 = M1_y ux + K1_y vx, s2 = M1_y vx
  for (int li = t; li < L; li += 64) {
    const int base = li % Q + L * (li / Q);
    line_apply<Q>(a.M1, ux, s1, base, Q);
    line_apply<Q>(a.K1, vx, x, base, Q);      // x is free again: holds K1_y vx
    line_apply<Q>(a.M1, vx, s2, base, Q);
  }
  __syncthreads();
  for (int l = t; l < MC; l += 64) s1[l] += x[l];
  __syncthreads();
  // z direction (base = a + Q b, stride Q^2): y = M1_z s1 + K1_z s2
  for (int li = t; li < L; li += 64) {
    line_apply<Q>(a.M1, s1, ux, li, L);
    line_apply<Q>(a.K1, s2, vx, li, L);
  }
  __syncthreads();
  for (int l = t; l < MC; l += 64) {
    const int nd = node[l];
    atomicAdd(a.q + nd, a.dscale[nd] * (ux[l] + vx[l]));
  }
}

}  // namespace

hipError_t launch_stiffness(const double* u, const double* dscale, double* q, int p, int nc, const double* K1,
                            const double* M1, hipStream_t s) {
  StiffArgs a{};
  a.u = u;
  a.dscale = dscale;
  a.q = q;
  a.nc = nc;
  a.n = nc * p;
  const int Q = p + 1;
  for (int i = 0; i < Q * Q; ++i) {
    a.K1[i] = K1[i];
    a.M1[i] = M1[i];
  }
  const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(nc) * nc * nc)), block(64);
  switch (p) {
    case 2: hipLaunchKernelGGL(stiffness_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(stiffness_kernel<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(stiffness_kernel<4>, grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL(stiffness_kernel<5>, grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL(stiffness_kernel<6>, grid, block, 0, s, a); break;
    case 7: hipLaunchKernelGGL(stiffness_kernel<7>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

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
