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
      for (; c + 112 < cn; c += 128) {  // eight loads in flight per lane
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = xr[c + 16 * u];
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          s0 = fma(ws[c + 16 * u] * x[u], x[u], s0);
          s1 = fma(ws[c + 16 * u + 16] * x[u + 1], x[u + 1], s1);
        }
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
  double eo[64];       // even-odd split of l_a(g_q), see interp_line
};

// One line of the tensor-product interpolation, out_q = sum_s I[q][s] v_s
// with I[q][s] = l_s(g_q).  The GLL nodes and the Gauss points are both
// symmetric about the cell centre, so I[Q-1-q][Q-1-s] = I[q][s] and the
// product splits into even and odd parts (H = floor(Q/2), m = H the middle
// index when Q is odd):
//   e_s = v_s + v_{Q-1-s},  d_s = v_s - v_{Q-1-s}            (s < H)
//   A_q = sum_s E[q][s] e_s (+ I[q][m] v_m),  B_q = sum_s O[q][s] d_s
//   out_q = A_q + B_q,  out_{Q-1-q} = A_q - B_q                 (q < H)
//   out_m = sum_s I[m][s] e_s + I[m][m] v_m
// with E, O = (I[q][s] +- I[q][Q-1-s]) / 2: 2H^2 + 2H + 1 coefficients
// (they stay in scalar registers) and about 3/4 of the multiply-adds.
// Table layout: E at q*H + s, O at H*H + q*H + s, I[q][m] at 2H*H + q,
// I[m][s] at 2H*H + H + s, I[m][m] at 2H*H + 2H.
template <int Q>
__device__ __forceinline__ void interp_line(const QuadArgs& a, const double (&v)[Q], double (&o)[Q]) {
  constexpr int H = Q / 2;
  constexpr bool ODD = (Q & 1) != 0;
  double e[H], d[H];
#pragma unroll
  for (int s = 0; s < H; ++s) {
    e[s] = v[s] + v[Q - 1 - s];
    d[s] = v[s] - v[Q - 1 - s];
  }
#pragma unroll
  for (int q = 0; q < H; ++q) {
    double A = 0.0, B = 0.0;
#pragma unroll
    for (int s = 0; s < H; ++s) {
      A = fma(a.eo[q * H + s], e[s], A);
      B = fma(a.eo[H * H + q * H + s], d[s], B);
    }
    if constexpr (ODD) A = fma(a.eo[2 * H * H + q], v[H], A);
    o[q] = A + B;
    o[Q - 1 - q] = A - B;
  }
  if constexpr (ODD) {
    double m = a.eo[2 * H * H + 2 * H] * v[H];
#pragma unroll
    for (int s = 0; s < H; ++s) m = fma(a.eo[2 * H * H + H + s], e[s], m);
    o[H] = m;
  }
}

// Waves per workgroup for order P: 4 line groups of 16 columns per wave,
// chosen so that the (p+1)^2 lines of a pass split into whole rounds with
// little idle: 9, 16, 25, 36, 49, 64 lines over 12, 16, 28, 36, 28, 32 groups.
template <int P>
constexpr int quad_waves() {
  return P == 2 ? 3 : P == 3 ? 4 : P == 4 ? 7 : P == 5 ? 9 : P == 6 ? 7 : 8;
}

// One workgroup per cell; 16 real columns per tile.  The gather of the next
// tile is issued into registers before the three interpolation passes of
// the current one, so its latency hides behind them.
template <int P>
__global__ __launch_bounds__(64 * quad_waves<P>()) __attribute__((amdgpu_waves_per_eu(P == 6 ? 4 : 1)))
void density_quad_kernel(QuadArgs a) {
  constexpr int Q = P + 1, MC = Q * Q * Q, CT = 16, LINES = Q * Q;
  constexpr int NT = 64 * quad_waves<P>(), NG = NT / CT;  // threads, line groups
  constexpr int IT = (LINES + NG - 1) / NG;               // lines per thread per pass
  constexpr int GI = (MC + NG - 1) / NG;                  // gathered rows per thread
  __shared__ double buf[MC * CT];                         // [local node][column]
  __shared__ double sc[MC];
  __shared__ int32_t node[MC];
  const int tid = threadIdx.x;
  const int col = tid & (CT - 1), grp = tid / CT;
  const int64_t e = blockIdx.x;
  const int cx = static_cast<int>(e % a.nc), cy = static_cast<int>((e / a.nc) % a.nc),
            cz = static_cast<int>(e / (static_cast<int64_t>(a.nc) * a.nc));
  for (int l = tid; l < MC; l += NT) {
    const int ax = l % Q, ay = (l / Q) % Q, az = l / (Q * Q);
    const int gx = (cx * P + ax) % a.n, gy = (cy * P + ay) % a.n, gz = (cz * P + az) % a.n;
    const int nd = gx + a.n * (gy + a.n * gz);
    node[l] = nd;
    sc[l] = a.dscale[nd];
  }
  __syncthreads();
  double acc[IT][Q];
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[it][q] = 0.0;

  // Columns past the block read column 0 (in bounds) and count as zero.  The
  // prefetch is unconditional (the last tile fetches column data it does not
  // use) so that no branch makes the compiler wait for it early.
  // gathered row i of this thread is local node min(grp + NG i, MC - 1)
  double g[GI], wn;
  {
    const int cs = col < a.ncr ? col : 0;
#pragma unroll
    for (int i = 0; i < GI; ++i)
      g[i] = a.X[static_cast<int64_t>(node[min(grp + NG * i, MC - 1)]) * a.ld + cs];
    wn = a.w[cs >> a.wshift];
  }
  for (int c0 = 0; c0 < a.ncr; c0 += CT) {
    const bool cok = c0 + col < a.ncr;
    const double wc = cok ? wn : 0.0;
    __syncthreads();  // scale table ready / previous tile fully consumed
#pragma unroll
    for (int i = 0; i < GI; ++i) {
      const int l = grp + NG * i;
      if (l < MC) buf[l * CT + col] = cok ? g[i] * sc[l] : 0.0;
    }
    __syncthreads();
    {  // prefetch the next tile
      const int cn = c0 + CT + col;
      const int cs = cn < a.ncr ? cn : 0;
#pragma unroll
      for (int i = 0; i < GI; ++i)
        g[i] = a.X[static_cast<int64_t>(node[min(grp + NG * i, MC - 1)]) * a.ld + cs];
      wn = a.w[cs >> a.wshift];
    }
    // axis x: line li = (b, c), elements li*Q + s
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int li = it * NG + grp;
      if (li < LINES) {
        double v[Q], o[Q];
#pragma unroll
        for (int s = 0; s < Q; ++s) v[s] = buf[(li * Q + s) * CT + col];
        interp_line<Q>(a, v, o);
#pragma unroll
        for (int q = 0; q < Q; ++q) buf[(li * Q + q) * CT + col] = o[q];
      }
    }
    __syncthreads();
    // axis y: line li = (a, c), elements (li % Q) + Q*Q*(li / Q) + Q*s
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int li = it * NG + grp;
      if (li < LINES) {
        const int base = li % Q + Q * Q * (li / Q);
        double v[Q], o[Q];
#pragma unroll
        for (int s = 0; s < Q; ++s) v[s] = buf[(base + Q * s) * CT + col];
        interp_line<Q>(a, v, o);
#pragma unroll
        for (int q = 0; q < Q; ++q) buf[(base + Q * q) * CT + col] = o[q];
      }
    }
    __syncthreads();
    // axis z: line li = (a, b), elements li + Q*Q*s; weighted squares kept
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int li = it * NG + grp;
      if (li < LINES) {
        double v[Q], o[Q];
#pragma unroll
        for (int s = 0; s < Q; ++s) v[s] = buf[(li + Q * Q * s) * CT + col];
        interp_line<Q>(a, v, o);
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[it][q] = fma(wc * o[q], o[q], acc[it][q]);
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
      const int li = it * NG + grp;
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
  // mirror-symmetrise the table (exact in the mathematics, not in the
  // rounded nodes), then split it into even and odd parts
  const int Q = d.p + 1, H = Q / 2, qq = Q * Q;
  double I[64];
  for (int i = 0; i < qq; ++i) I[i] = 0.5 * (d.interp[i] + d.interp[qq - 1 - i]);
  for (int q = 0; q < H; ++q) {
    for (int s = 0; s < H; ++s) {
      a.eo[q * H + s] = 0.5 * (I[q * Q + s] + I[q * Q + Q - 1 - s]);
      a.eo[H * H + q * H + s] = 0.5 * (I[q * Q + s] - I[q * Q + Q - 1 - s]);
    }
    if (Q & 1) a.eo[2 * H * H + q] = I[q * Q + H];
  }
  if (Q & 1) {
    for (int s = 0; s < H; ++s) a.eo[2 * H * H + H + s] = I[H * Q + s];
    a.eo[2 * H * H + 2 * H] = I[H * Q + H];
  }
  const dim3 grid(static_cast<unsigned>(d.E));
#define CHFSI_DQ(P) \
  hipLaunchKernelGGL(density_quad_kernel<P>, grid, dim3(64 * quad_waves<P>()), 0, s, a)
  switch (d.p) {
    case 2: CHFSI_DQ(2); break;
    case 3: CHFSI_DQ(3); break;
    case 4: CHFSI_DQ(4); break;
    case 5: CHFSI_DQ(5); break;
    case 6: CHFSI_DQ(6); break;
    case 7: CHFSI_DQ(7); break;
    default: return hipErrorInvalidValue;
  }
#undef CHFSI_DQ
  return hipGetLastError();
}

}  // namespace chfsi
