// Kernels of the self-consistent field loop (Section 3, Algorithm 1): the
// stiffness operator of the Hartree problem applied to one vector by sum
// factorisation, the iterations of its preconditioned CG with the scalars
// kept on the device, and single passes over M values for its right-hand
// side, the Jacobi preconditioner, the effective potential with LDA
// exchange and the weighted vectors of the mixing.
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
  const int32_t* cells;  // deterministic assembly: the cells of one colour class (null: all)
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
  const int64_t e = a.cells ? a.cells[blockIdx.x] : blockIdx.x;
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
                            const double* M1, hipStream_t s, const int32_t* cells, int ncell) {
  StiffArgs a{};
  a.u = u;
  a.dscale = dscale;
  a.q = q;
  a.cells = cells;
  a.nc = nc;
  a.n = nc * p;
  const int Q = p + 1;
  for (int i = 0; i < Q * Q; ++i) {
    a.K1[i] = K1[i];
    a.M1[i] = M1[i];
  }
  const dim3 grid(static_cast<unsigned>(cells ? ncell : static_cast<int64_t>(nc) * nc * nc)), block(64);
  if (grid.x == 0) return hipSuccess;
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

namespace {

// ---- preconditioned CG with its scalars on the device ------------------------
// sc[0] = r.z, sc[1] = p.q, sc[2] = r.r, sc[3] = z.n, sc[4] = r.z (new),
// sc[5] = |n|^2 (n = M^1/2 1, the null vector); dot products accumulate by
// one atomic add per block, or, for deterministic results, each block
// stores its partial sum of scalar k at part[k * kCgMaxBlocks + block] and
// one block sums them in a fixed order (cg_sum_kernel).

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return t;   // valid in thread 0
}

constexpr int kCgMaxBlocks = 256;

// block partial v of scalar k: added into sc[k], or stored for cg_sum_kernel
__device__ __forceinline__ void put_partial(double* sc, double* part, int k, double v) {
  if (threadIdx.x != 0) return;
  if (part) part[k * kCgMaxBlocks + blockIdx.x] = v;
  else atomicAdd(sc + k, v);
}

// sc[k] = sum of the nb partials of scalar k, for k in [k0, k0 + cnt), in
// one fixed order (one block)
__global__ void __launch_bounds__(256) cg_sum_kernel(const double* __restrict__ part, double* __restrict__ sc,
                                                     int k0, int cnt, int nb) {
  for (int k = k0; k < k0 + cnt; ++k) {
    const double v = block_sum(threadIdx.x < nb ? part[k * kCgMaxBlocks + threadIdx.x] : 0.0);
    if (threadIdx.x == 0) sc[k] = v;
  }
}

__global__ void __launch_bounds__(256) cg_pq_kernel(const double* __restrict__ p, const double* __restrict__ q,
                                                    double* __restrict__ sc, double* __restrict__ part, int64_t n) {
  double v = 0.0;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) v += p[i] * q[i];
  v = block_sum(v);
  put_partial(sc, part, 1, v);
}

// u += a p, r -= a q, z = r / kd; sums r.r, z.n, r.n
__global__ void __launch_bounds__(256) cg_update_kernel(double* __restrict__ u, double* __restrict__ r,
                                                        double* __restrict__ z, const double* __restrict__ p,
                                                        const double* __restrict__ q, const double* __restrict__ kd,
                                                        const double* __restrict__ nv, double* __restrict__ sc,
                                                        double* __restrict__ part, int64_t n) {
  const double pq = sc[1];
  const double al = pq > 0.0 ? sc[0] / pq : 0.0;
  double rr = 0.0, zn = 0.0;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    u[i] += al * p[i];
    const double ri = r[i] - al * q[i];
    r[i] = ri;
    const double zi = ri / kd[i];
    z[i] = zi;
    rr += ri * ri;
    zn += zi * nv[i];
  }
  rr = block_sum(rr);
  put_partial(sc, part, 2, rr);
  zn = block_sum(zn);
  put_partial(sc, part, 3, zn);
}

// z -= (z.n / n.n) n; sum r.z
__global__ void __launch_bounds__(256) cg_project_kernel(const double* __restrict__ r, double* __restrict__ z,
                                                         const double* __restrict__ nv, double* __restrict__ sc,
                                                         double* __restrict__ part, int64_t n) {
  const double c = sc[3] / sc[5];
  double rz = 0.0;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const double zi = z[i] - c * nv[i];
    z[i] = zi;
    rz += r[i] * zi;
  }
  rz = block_sum(rz);
  put_partial(sc, part, 4, rz);
}

// p = z + (rz_new / rz) p
__global__ void __launch_bounds__(256) cg_direction_kernel(const double* __restrict__ z, double* __restrict__ p,
                                                           const double* __restrict__ sc, int64_t n) {
  const double be = sc[0] > 0.0 ? sc[4] / sc[0] : 0.0;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) p[i] = z[i] + be * p[i];
}

// scalar bookkeeping between iterations: keep r.r of iteration `it`, move the
// new r.z into place, clear the sums
__global__ void cg_scalars_kernel(double* __restrict__ sc, double* __restrict__ hist, int it) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    hist[it] = sc[2];
    sc[0] = sc[4];
    sc[1] = 0.0;
    sc[2] = 0.0;
    sc[3] = 0.0;
    sc[4] = 0.0;
  }
}

// at most one block per compute unit: every block adds its partial sums
// into the same few scalars, and those atomics serialise in L2
unsigned cg_grid(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return static_cast<unsigned>(b < kCgMaxBlocks ? b : kCgMaxBlocks);
}

}  // namespace

hipError_t launch_cg_iteration(double* u, double* r, double* z, double* p, const double* q, const double* kd,
                               const double* nv, double* sc, double* hist, int it, int64_t n, hipStream_t s,
                               double* part) {
  const dim3 g(cg_grid(n)), b(256);
  const int nb = static_cast<int>(g.x);
  hipLaunchKernelGGL(cg_pq_kernel, g, b, 0, s, p, q, sc, part, n);
  if (part) hipLaunchKernelGGL(cg_sum_kernel, dim3(1), b, 0, s, part, sc, 1, 1, nb);
  hipLaunchKernelGGL(cg_update_kernel, g, b, 0, s, u, r, z, p, q, kd, nv, sc, part, n);
  if (part) hipLaunchKernelGGL(cg_sum_kernel, dim3(1), b, 0, s, part, sc, 2, 2, nb);
  hipLaunchKernelGGL(cg_project_kernel, g, b, 0, s, r, z, nv, sc, part, n);
  if (part) hipLaunchKernelGGL(cg_sum_kernel, dim3(1), b, 0, s, part, sc, 4, 1, nb);
  hipLaunchKernelGGL(cg_direction_kernel, g, b, 0, s, z, p, sc, n);
  hipLaunchKernelGGL(cg_scalars_kernel, dim3(1), dim3(64), 0, s, sc, hist, it);
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
