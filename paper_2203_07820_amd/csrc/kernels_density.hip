// Electron density from a block of Loewdin-basis vectors (Section 3.2, the
// density-computation algorithm; density definition of Section 2.1).
//
// rho(x) = sum_c w_c |psi^_c(x)|^2 with psi^ = M^-1/2 psi~ interpolated by the
// FE basis.  The weights carry the occupations: 2 f_i for Ritz vectors, or in
// the spectrum-split form 2 for an orthonormal basis of the filtered space
// plus 2 (f_i - 1) for the fractionally occupied Ritz vectors (two calls that
// accumulate into the same rho).
//
// Two evaluation sets:
//  * nodes: the FE basis is nodal, so rho at node j is
//    M_jj^-1 sum_c w_c |X_jc|^2.  Pure streaming over X: one wave takes four
//    rows per step, 16 lanes per row, weights staged in LDS.
//  * Gauss points of every cell ((p+1)^3 per cell, the rule the operator is
//    integrated with): the cell's nodal values are interpolated with the
//    tensor-product Lagrange basis, applied one axis at a time (three passes
//    of a (p+1) x (p+1) matrix over the cell's lines, in LDS) instead of one
//    dense mcell x mcell product: 3 (p+1)^4 instead of (p+1)^6 multiply-adds
//    per column, which leaves the kernel bound by the gather of X.  One
//    workgroup per cell walks all column tiles and keeps the weighted squares
//    in registers, so every rho entry is written once, without atomics.
//
// X is read as a real view: complex data is interleaved (re, im) and both
// parts carry the weight of their column (wshift = 1), which sums
// re^2 + im^2 = |psi|^2.
#include "internal.h"

namespace chfsi {
namespace {

constexpr int kThreads = 256;
constexpr int kWChunk = 2048;  // real-view columns of weights staged per round

__global__ __launch_bounds__(kThreads) void density_nodes_kernel(const double* __restrict__ X, int64_t ld, int ncr,
                                                                 int wshift, const double* __restrict__ w,
                                                                 const double* __restrict__ dscale,
                                                                 double* __restrict__ rho, int64_t M, int accumulate) {
  __shared__ double ws[kWChunk];
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, sub = lane & 15;
  const int64_t wave = static_cast<int64_t>(blockIdx.x) * (kThreads / 64) + (threadIdx.x >> 6);
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * (kThreads / 64);
  for (int c0 = 0; c0 < ncr; c0 += kWChunk) {
    const int cn = min(kWChunk, ncr - c0);
    __syncthreads();
    for (int i = threadIdx.x; i < cn; i += kThreads) ws[i] = w[(c0 + i) >> wshift];
    __syncthreads();
    const bool add = accumulate || c0 > 0;
    for (int64_t rq = wave * 4; rq < M; rq += nwaves * 4) {
      const int64_t r = rq + g;
      const bool live = r < M;
      // rows past the end read the last row (in bounds) and store nothing
      const double* xr = X + (live ? r : M - 1) * ld + c0;
      double s0 = 0.0, s1 = 0.0;
      int c = sub;
      for (; c + 48 < cn; c += 64) {
        const double x0 = xr[c], x1 = xr[c + 16], x2 = xr[c + 32], x3 = xr[c + 48];
        s0 = fma(ws[c] * x0, x0, s0);
        s1 = fma(ws[c + 16] * x1, x1, s1);
        s0 = fma(ws[c + 32] * x2, x2, s0);
        s1 = fma(ws[c + 48] * x3, x3, s1);
      }
      for (; c < cn; c += 16) {
        const double x0 = xr[c];
        s0 = fma(ws[c] * x0, x0, s0);
      }
      double s = s0 + s1;
      s += __shfl_xor(s, 8, 16);
      s += __shfl_xor(s, 4, 16);
      s += __shfl_xor(s, 2, 16);
      s += __shfl_xor(s, 1, 16);
      if (live && sub == 0) {
        const double d = dscale[r];
        const double v = d * d * s;
        rho[r] = add ? rho[r] + v : v;
      }
    }
  }
}

struct QuadArgs {
  const double* X;
  int64_t ld;          // real view
  int ncr;             // real-view columns
  int wshift;
  const double* w;     // ncols weights
  const double* dscale;
  double* rho;         // E x (p+1)^3
  int nc, n;           // cells and nodes per side
  int accumulate;
  double interp[64];   // interp[q * (p+1) + a] = l_a(g_q)
};

// One workgroup per cell; 16 real columns per tile, 16 line groups.
template <int P>
__global__ __launch_bounds__(kThreads) void density_quad_kernel(QuadArgs a) {
  constexpr int Q = P + 1, MC = Q * Q * Q, CT = 16, LINES = Q * Q;
  constexpr int IT = (LINES * CT + kThreads - 1) / kThreads;  // lines per thread per pass
  __shared__ double buf[MC * CT];                              // [local node][column]
  __shared__ int32_t node[MC];
  __shared__ double sc[MC];
  const int tid = threadIdx.x;
  const int col = tid & (CT - 1), grp = tid >> 4;
  const int64_t e = blockIdx.x;
  const int cx = static_cast<int>(e % a.nc), cy = static_cast<int>((e / a.nc) % a.nc),
            cz = static_cast<int>(e / (static_cast<int64_t>(a.nc) * a.nc));
  for (int l = tid; l < MC; l += kThreads) {
    const int ax = l % Q, ay = (l / Q) % Q, az = l / (Q * Q);
    const int gx = (cx * P + ax) % a.n, gy = (cy * P + ay) % a.n, gz = (cz * P + az) % a.n;
    const int nd = gx + a.n * (gy + a.n * gz);
    node[l] = nd;
    sc[l] = a.dscale[nd];
  }
  double acc[IT][Q];
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[it][q] = 0.0;

  for (int c0 = 0; c0 < a.ncr; c0 += CT) {
    const int cc = c0 + col;
    const bool cok = cc < a.ncr;
    const double wc = cok ? a.w[cc >> a.wshift] : 0.0;
    __syncthreads();  // tables ready / previous tile fully consumed
    for (int l = grp; l < MC; l += kThreads / CT)
      buf[l * CT + col] = cok ? a.X[static_cast<int64_t>(node[l]) * a.ld + cc] * sc[l] : 0.0;
    __syncthreads();
    // axis x: line li = (b, c), elements li*Q + s
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int li = it * (kThreads / CT) + grp;
      if (li < LINES) {
        double v[Q];
#pragma unroll
        for (int s = 0; s < Q; ++s) v[s] = buf[(li * Q + s) * CT + col];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          double o = 0.0;
#pragma unroll
          for (int s = 0; s < Q; ++s) o = fma(a.interp[q * Q + s], v[s], o);
          buf[(li * Q + q) * CT + col] = o;
        }
      }
    }
    __syncthreads();
    // axis y: line li = (a, c), elements (li % Q) + Q*Q*(li / Q) + Q*s
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int li = it * (kThreads / CT) + grp;
      if (li < LINES) {
        const int base = li % Q + Q * Q * (li / Q);
        double v[Q];
#pragma unroll
        for (int s = 0; s < Q; ++s) v[s] = buf[(base + Q * s) * CT + col];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          double o = 0.0;
#pragma unroll
          for (int s = 0; s < Q; ++s) o = fma(a.interp[q * Q + s], v[s], o);
          buf[(base + Q * q) * CT + col] = o;
        }
      }
    }
    __syncthreads();
    // axis z: line li = (a, b), elements li + Q*Q*s; weighted squares kept
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int li = it * (kThreads / CT) + grp;
      if (li < LINES) {
        double v[Q];
#pragma unroll
        for (int s = 0; s < Q; ++s) v[s] = buf[(li + Q * Q * s) * CT + col];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          double o = 0.0;
#pragma unroll
          for (int s = 0; s < Q; ++s) o = fma(a.interp[q * Q + s], v[s], o);
          acc[it][q] = fma(wc * o, o, acc[it][q]);
        }
      }
    }
  }
  // sum over the 16 columns of the tile (lanes of one line group)
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      double s = acc[it][q];
      s += __shfl_xor(s, 8, 16);
      s += __shfl_xor(s, 4, 16);
      s += __shfl_xor(s, 2, 16);
      s += __shfl_xor(s, 1, 16);
      acc[it][q] = s;
    }
  if (col == 0) {
    double* out = a.rho + e * MC;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int li = it * (kThreads / CT) + grp;
      if (li < LINES) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int idx = li + Q * Q * q;
          out[idx] = a.accumulate ? out[idx] + acc[it][q] : acc[it][q];
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_density(const DensityLaunch& d, hipStream_t s) {
  const int wshift = d.cplx ? 1 : 0;
  const int ncr = d.ncols << wshift;
  const int64_t ldr = d.ld << wshift;
  if (d.points == 0) {
    const int64_t quads = (d.M + 15) / 16;  // four rows per wave, four waves per block
    const int grid = static_cast<int>(std::min<int64_t>(quads, 8192));
    hipLaunchKernelGGL(density_nodes_kernel, dim3(grid), dim3(kThreads), 0, s, d.X, ldr, ncr, wshift, d.w, d.dscale,
                       d.rho, d.M, d.accumulate);
    return hipGetLastError();
  }
  QuadArgs a{};
  a.X = d.X;
  a.ld = ldr;
  a.ncr = ncr;
  a.wshift = wshift;
  a.w = d.w;
  a.dscale = d.dscale;
  a.rho = d.rho;
  a.nc = d.nc;
  a.n = d.nc * d.p;
  a.accumulate = d.accumulate;
  const int q = d.p + 1;
  for (int i = 0; i < q * q; ++i) a.interp[i] = d.interp[i];
  const dim3 grid(static_cast<unsigned>(d.E)), block(kThreads);
  switch (d.p) {
    case 2: hipLaunchKernelGGL(density_quad_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(density_quad_kernel<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(density_quad_kernel<4>, grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL(density_quad_kernel<5>, grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL(density_quad_kernel<6>, grid, block, 0, s, a); break;
    case 7: hipLaunchKernelGGL(density_quad_kernel<7>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace chfsi
