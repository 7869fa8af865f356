// Tall-skinny FP64 subspace kernels of the Rayleigh-Ritz step (DFT-FE 1.0,
// Section 4.4 and Algorithm 2): the overlap / projected-Hamiltonian Gram
// products A = X^H Y (lower triangle only, split over rows with a
// deterministic two-phase reduction, the single-GPU counterpart of the
// blocked, all-reduced N x B_v slabs), the subspace rotation X' = X Z, and
// residual column norms.  Complex data is handled through its real view
// (interleaved re, im): X^H Y and X Z become real products of twice the width
// whose entries are recombined, which costs exactly the complex flop count.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace chfsi {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register i holds D[4 i + l / 16][l % 16].
__device__ __forceinline__ d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int acc_row(int lane, int i) { return 4 * i + lane / 16; }

// The same products for FP64 and FP32 data.  v_mfma_f32_16x16x4f32 takes its
// operands in the same lanes as the f64 instruction; its accumulator
// register i holds D[4 (l / 16) + i][l % 16].
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using Acc = d4;
  static __device__ __forceinline__ Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + lane / 16; }
};
template <> struct Mfma<float> {
  using Acc = f4;
  static __device__ __forceinline__ Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane / 16) + i; }
};

// ---- Gram: partial[chunk] tile (I, J), I >= J, of X^T Y --------------------
// One workgroup computes a 128 x 128 tile over the rows of one chunk; 4 waves
// of 64 x 64 (4 x 4 MFMA tiles).  In a 4-row k step, lanes 16 q .. 16 q + 15
// read 16 consecutive columns of row 4 s + q, which is both the A operand
// (X^T) and the B operand (Y) layout of the f64 MFMA, so the fragments go
// straight from memory into registers: buffer loads from the chunk's first
// row, the row offset in the lane's voffset (clamped to the chunk, tail rows
// zeroed at use), the four 16-column groups in the instruction offset.
// Loads run two k steps ahead of the MFMAs; no LDS, no barriers.
constexpr int kGT = 128;  // Gram tile
constexpr int kGramStages = 3;   // register stages of the Gram pipeline (loads GS - 1 steps ahead)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, 0x00020000);
}
template <typename T, int OFF>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int voff);
template <int OFF>
__device__ __forceinline__ double bload64(__amdgpu_buffer_rsrc_t r, int voff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff + OFF, 0, 0));
}
template <int OFF>
__device__ __forceinline__ float bload32(__amdgpu_buffer_rsrc_t r, int voff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff + OFF, 0, 0));
}
template <typename T, int G>   // 16-column group G of the lane's row
__device__ __forceinline__ T bload_group(__amdgpu_buffer_rsrc_t r, int voff) {
  if constexpr (sizeof(T) == 8) return bload64<G * 128>(r, voff);
  else return bload32<G * 64>(r, voff);
}

template <typename T, int GS>
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2)))
gram_kernel(const T* __restrict__ X, int64_t ldx, const T* __restrict__ Y, int64_t ldy,
            int64_t M, int n, int64_t rows_per_chunk, int npad, double* __restrict__ part, int64_t offx,
            int64_t offy) {
  const int t = blockIdx.x;
  // lower-triangular tile index -> (I, J)
  int I = static_cast<int>((sqrt(8.0 * t + 1.0) - 1.0) / 2.0);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int chunk = blockIdx.y;
  const int64_t m0 = chunk * rows_per_chunk;
  int64_t m1 = m0 + rows_per_chunk;
  if (m1 > M) m1 = M;
  const int nrows = static_cast<int>(m1 - m0);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wi = (wave / 2) * 64, wj = (wave % 2) * 64;
  using Acc = typename Mfma<T>::Acc;
  Acc acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = Acc{0, 0, 0, 0};
  // per-lane column of the first 16-column group (the others are +16 k).
  // Columns at or beyond n belong to the tile's padding, which is never read
  // back: what they load (the rest of the row, the next row, or zero past the
  // end of the chunk, where the buffer range check returns 0) does not matter.
  const int ci = I * kGT + wi + lane % 16;
  const int cj = J * kGT + wj + lane % 16;
  const int64_t nr = nrows > 0 ? nrows : 0;
  // X and Y may start offx / offy columns into their rows (a column slice):
  // the ranges then end offx / offy elements before the last row's end, so
  // the padding columns of the last chunk never reach past the allocation
  const int64_t ex = nr > 0 ? (nr * ldx < (M - m0) * ldx - offx ? nr * ldx : (M - m0) * ldx - offx) : 0;
  const int64_t ey = nr > 0 ? (nr * ldy < (M - m0) * ldy - offy ? nr * ldy : (M - m0) * ldy - offy) : 0;
  const __amdgpu_buffer_rsrc_t rx = rsrc(X + (nr > 0 ? m0 * ldx : 0), static_cast<uint32_t>(ex * sizeof(T)));
  const __amdgpu_buffer_rsrc_t ry = rsrc(Y + (nr > 0 ? m0 * ldy : 0), static_cast<uint32_t>(ey * sizeof(T)));
  const int KS = nrows > 0 ? (nrows + 3) / 4 : 0;   // every chunk still writes its tile
  auto load = [&](T (&xv)[4], T (&yv)[4], int s) {
    const int row = min(4 * s + lane / 16, nrows - 1);
    const int vx = (row * static_cast<int>(ldx) + ci) * static_cast<int>(sizeof(T));
    const int vy = (row * static_cast<int>(ldy) + cj) * static_cast<int>(sizeof(T));
    xv[0] = bload_group<T, 0>(rx, vx);
    xv[1] = bload_group<T, 1>(rx, vx);
    xv[2] = bload_group<T, 2>(rx, vx);
    xv[3] = bload_group<T, 3>(rx, vx);
    yv[0] = bload_group<T, 0>(ry, vy);
    yv[1] = bload_group<T, 1>(ry, vy);
    yv[2] = bload_group<T, 2>(ry, vy);
    yv[3] = bload_group<T, 3>(ry, vy);
  };
  auto compute = [&](const T (&xin)[4], const T (&yin)[4], int s) {
    T xv[4], yv[4];
    const bool ok = 4 * s + lane / 16 < nrows;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      xv[a] = ok ? xin[a] : T(0);
      yv[a] = ok ? yin[a] : T(0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::mma(xv[a], yv[b], acc[a][b]);
  };
  // GS register stages with fixed roles (the loop is unrolled by GS; three
  // by default: four or five measured no faster): the rows of step
  // s + GS - 1 are in flight while step s multiplies.  A copy between stages
  // would make the compiler wait for the loads in flight into the source.
  // Loads past the last step read the chunk's last row (the row index is
  // clamped) and the steps past KS contribute zero.
  T xq[GS][4], yq[GS][4];
  if (KS > 0) {
#pragma unroll
    for (int j = 0; j < GS - 1; ++j) load(xq[j], yq[j], j);
  }
  for (int s = 0; s < KS; s += GS) {
#pragma unroll
    for (int j = 0; j < GS; ++j) {
      load(xq[(j + GS - 1) % GS], yq[(j + GS - 1) % GS], s + j + GS - 1);
      compute(xq[j], yq[j], s + j);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  double* out = part + static_cast<int64_t>(chunk) * npad * npad;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = I * kGT + wi + a * 16 + Mfma<T>::row(lane, i);
        const int col = J * kGT + wj + b * 16 + lane % 16;
        out[static_cast<int64_t>(row) * npad + col] = static_cast<double>(acc[a][b][i]);
      }
}

__global__ void gram_reduce_kernel(const double* __restrict__ part, int nchunks, int n, int npad,
                                   double* __restrict__ G, int64_t ldg) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int i = static_cast<int>(idx / n), j = static_cast<int>(idx % n);
  if (i / kGT < j / kGT) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(static_cast<int64_t>(c) * npad + i) * npad + j];
  G[static_cast<int64_t>(i) * ldg + j] = s;
}

// Real symmetric result from the lower entries: S[i][j] = G[max][min].
__global__ void sym_from_lower_kernel(const double* __restrict__ G, int64_t ldg, double* __restrict__ S,
                                      int n) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int i = static_cast<int>(idx / n), j = static_cast<int>(idx % n);
  const int a = i > j ? i : j, b = i > j ? j : i;
  S[idx] = G[static_cast<int64_t>(a) * ldg + b];
}

// Complex Hermitian S (n x n, column-major interleaved) from the real-view
// Gram G2 (2n x 2n) of interleaved X, Y:
// S_ij = (G[2i][2j] + G[2i+1][2j+1]) + i (G[2i][2j+1] - G[2i+1][2j]) for
// i >= j, S_ji = conj(S_ij).
__global__ void gram_combine_complex_kernel(const double* __restrict__ G, int64_t ldg,
                                            double* __restrict__ S, int n) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int i = static_cast<int>(idx / n), j = static_cast<int>(idx % n);
  const int a = i > j ? i : j, b = i > j ? j : i;
  const double g00 = G[static_cast<int64_t>(2 * a) * ldg + 2 * b];
  const double g11 = G[static_cast<int64_t>(2 * a + 1) * ldg + 2 * b + 1];
  const double g01 = G[static_cast<int64_t>(2 * a) * ldg + 2 * b + 1];
  const double g10 = G[static_cast<int64_t>(2 * a + 1) * ldg + 2 * b];
  const double re = g00 + g11;
  double im = g01 - g10;
  if (i < j) im = -im;   // conjugate for the upper triangle
  if (i == j) im = 0.0;
  // column-major: element (i, j) at i + j n
  const int64_t o = (static_cast<int64_t>(i) + static_cast<int64_t>(j) * n) * 2;
  S[o] = re;
  S[o + 1] = im;
}

// ---- rotation C = X Z --------------------------------------------------------
// Workgroup tile 128 x 128, 4 waves of 64 x 64 (4 x 4 MFMA tiles: each A and
// B fragment read from LDS serves four MFMAs).  X rows are staged through
// LDS (the A operand needs 16 rows per fragment), Z through LDS as well; both
// double buffered, with the next 16-deep k chunk loaded into registers from
// global memory while the current one multiplies, so there is one barrier
// per chunk (64 MFMAs per wave) and the global latency overlaps the MFMAs.
// The two stages take 70 KB of LDS at FP64: two workgroups per CU.
// upper: Z is upper triangular, k stops at the tile's last column.
constexpr int kRM = 128;  // rows per workgroup
constexpr int kRN = 128;  // columns per workgroup
constexpr int kRK = 16;   // k per stage
constexpr int kZP = kRN + 8;  // padded LDS row of the Z stage

template <typename T>
__global__ void __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2)))
rotate_kernel(const T* __restrict__ X, int64_t ldx, const T* __restrict__ Z, int64_t ldz,
              T* __restrict__ C, int64_t ldc, int64_t M, int K, int N2, int upper) {
  __shared__ T xs[2][kRM][kRK + 1];
  __shared__ T zs[2][kRK][kZP];
  const int64_t r0 = blockIdx.x * static_cast<int64_t>(kRM);
  const int c0 = blockIdx.y * kRN;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wr = (wave / 2) * 64, wc = (wave % 2) * 64;
  using Acc = typename Mfma<T>::Acc;
  Acc acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = Acc{0, 0, 0, 0};
  int kend = K;
  if (upper && c0 + kRN < kend) kend = c0 + kRN;
  // loaders: X 128 rows x 16 k (8 per thread, 16 threads per row), Z 16 k x
  // 128 columns (8 per thread, one row per 128 threads); addresses clamped,
  // out-of-range values zeroed when stored to LDS
  const int xk = tid % kRK, xr = tid / kRK;
  const int zc = tid % kRN, zr = tid / kRN;
  T gx[8], gz[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      int64_t row = r0 + xr + 16 * i;
      row = row < M ? row : M - 1;
      int k = k0 + xk;
      k = k < K ? k : K - 1;
      gx[i] = X[row * ldx + k];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      int k = k0 + zr + 2 * i;
      k = k < K ? k : K - 1;
      int c = c0 + zc;
      c = c < N2 ? c : N2 - 1;
      gz[i] = Z[static_cast<int64_t>(k) * ldz + c];
    }
  };
  auto sstore = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bool ok = r0 + xr + 16 * i < M && k0 + xk < K;
      xs[buf][xr + 16 * i][xk] = ok ? gx[i] : T(0);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bool ok = k0 + zr + 2 * i < K && c0 + zc < N2;
      zs[buf][zr + 2 * i][zc] = ok ? gz[i] : T(0);
    }
  };
  if (kend > 0) {
    gload(0);
    sstore(0, 0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < kend; k0 += kRK) {
    const bool more = k0 + kRK < kend;
    if (more) gload(k0 + kRK);
#pragma unroll
    for (int ks = 0; ks < kRK / 4; ++ks) {
      const int kr = ks * 4 + lane / 16;
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = xs[buf][wr + a * 16 + lane % 16][kr];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = zs[buf][kr][wc + b * 16 + lane % 16];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::mma(av[a], bv[b], acc[a][b]);
    }
    if (more) sstore(buf ^ 1, k0 + kRK);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = r0 + wr + a * 16 + Mfma<T>::row(lane, i);
        const int col = c0 + wc + b * 16 + lane % 16;
        if (row < M && col < N2) C[row * ldc + col] = acc[a][b][i];
      }
}

// ---- residual column sums ------------------------------------------------
__global__ void __launch_bounds__(256)
resid_kernel(const double* __restrict__ HX, int64_t ldh, const double* __restrict__ X, int64_t ldx,
             const double* __restrict__ th, int64_t M, int ncols, int cplx, int64_t rows_per_chunk,
             double* __restrict__ part) {
  const int j = blockIdx.y * 256 + threadIdx.x;
  if (j >= ncols) return;
  const int64_t m0 = blockIdx.x * rows_per_chunk;
  int64_t m1 = m0 + rows_per_chunk;
  if (m1 > M) m1 = M;
  const double t = th[j];
  double s = 0.0;
  if (cplx) {
    for (int64_t r = m0; r < m1; ++r) {
      const double dr = HX[(r * ldh + j) * 2] - t * X[(r * ldx + j) * 2];
      const double di = HX[(r * ldh + j) * 2 + 1] - t * X[(r * ldx + j) * 2 + 1];
      s += dr * dr + di * di;
    }
  } else {
    for (int64_t r = m0; r < m1; ++r) {
      const double d = HX[r * ldh + j] - t * X[r * ldx + j];
      s += d * d;
    }
  }
  part[static_cast<int64_t>(blockIdx.x) * ncols + j] = s;
}

// ---- vector helpers --------------------------------------------------------
constexpr int kDotBlocks = 1024;

__global__ void __launch_bounds__(256)
dot_kernel(const double* __restrict__ x, const double* __restrict__ y, int64_t n, double* part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * 256)
    s += x[i] * y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, double* __restrict__ y,
                             int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

__global__ void transpose_kernel(const double* __restrict__ in, double* __restrict__ out, int n) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int i = static_cast<int>(idx / n), j = static_cast<int>(idx % n);
  out[static_cast<int64_t>(j) * n + i] = in[idx];
}

// out (cols x rows, ldo) = in^T, in rows x cols (ldi), row-major
__global__ void transpose_rect_kernel(const double* __restrict__ in, int64_t ldi, int rows, int cols,
                                      double* __restrict__ out, int64_t ldo) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(rows) * cols) return;
  const int i = static_cast<int>(idx / cols), j = static_cast<int>(idx % cols);
  out[static_cast<int64_t>(j) * ldo + i] = in[static_cast<int64_t>(i) * ldi + j];
}

// Splits the upper-triangular n x n Z (row-major, ldz): Zo = FP32 copy with
// the diagonal removed, d = the diagonal in FP64.
__global__ void split_diag_kernel(const double* __restrict__ Z, int64_t ldz, int n, float* __restrict__ Zo,
                                  double* __restrict__ d) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int i = static_cast<int>(idx / n), j = static_cast<int>(idx % n);
  const double z = Z[static_cast<int64_t>(i) * ldz + j];
  Zo[idx] = i == j ? 0.0f : static_cast<float>(z);
  if (i == j) d[i] = z;
}

// X[r][j] <- C[r][j] + d[j] X[r][j]   (C in FP32, X and d in FP64)
__global__ void add_scaled_cols_kernel(const float* __restrict__ C, int64_t ldc, const double* __restrict__ d,
                                       double* __restrict__ X, int64_t ldx, int64_t M, int n) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= M * n) return;
  const int64_t r = idx / n;
  const int j = static_cast<int>(idx % n);
  double* x = X + r * ldx + j;
  *x = static_cast<double>(C[r * ldc + j]) + d[j] * *x;
}

__global__ void zero_strict_lower_kernel(double* A, int n, int64_t lda) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(n) * n) return;
  const int i = static_cast<int>(idx / n), j = static_cast<int>(idx % n);
  if (i > j) A[static_cast<int64_t>(i) * lda + j] = 0.0;
}

// Real 2n1 x 2n2 expansion of a complex matrix Z (row-major interleaved,
// Z[k][j] at (k n2 + j)), or of the conjugate of a column-major upper
// Cholesky-inverse read as row-major, so that [re im] rows times it give the
// complex product.  mode 0: Z given row-major.  mode 1: src is column-major
// L^-1 (n1 = n2); Z = L^-H, i.e. Z[k][j] = conj(src[k n + j]) for k <= j,
// 0 below the diagonal.  mode 2: src is column-major Q (eigenvectors); Z = Q,
// Z[k][j] = src[k + j n].
__global__ void expand_complex_kernel(const double* __restrict__ src, int n1, int n2, int mode,
                                      double* __restrict__ Z2) {
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= static_cast<int64_t>(n1) * n2) return;
  const int k = static_cast<int>(idx / n2), j = static_cast<int>(idx % n2);
  double zr, zi;
  if (mode == 0) {
    zr = src[idx * 2];
    zi = src[idx * 2 + 1];
  } else if (mode == 1) {
    if (k > j) {
      zr = 0.0;
      zi = 0.0;
    } else {
      zr = src[idx * 2];
      zi = -src[idx * 2 + 1];
    }
  } else {
    const int64_t o = (static_cast<int64_t>(k) + static_cast<int64_t>(j) * n1) * 2;
    zr = src[o];
    zi = src[o + 1];
  }
  const int64_t ld = 2 * static_cast<int64_t>(n2);
  Z2[(2 * static_cast<int64_t>(k)) * ld + 2 * j] = zr;
  Z2[(2 * static_cast<int64_t>(k)) * ld + 2 * j + 1] = zi;
  Z2[(2 * static_cast<int64_t>(k) + 1) * ld + 2 * j] = -zi;
  Z2[(2 * static_cast<int64_t>(k) + 1) * ld + 2 * j + 1] = zr;
}

unsigned blocks_for(int64_t total, int per = 256) {
  return static_cast<unsigned>((total + per - 1) / per);
}

// Row chunks of the Gram products: about 1024 workgroups in all, at least
// 256 rows per chunk, and few enough rows that a chunk of the widest operand
// (ld doubles per row) spans less than 2^31 bytes (32-bit buffer offsets).
int gram_chunks(int64_t M, int n, int64_t ld) {
  const int nt = (n + kGT - 1) / kGT;
  const int ntiles = nt * (nt + 1) / 2;
  int64_t ch = (1024 + ntiles - 1) / ntiles;
  const int64_t max_ch = (M + 255) / 256;
  if (ch > max_ch) ch = max_ch;
  const int64_t max_rows = ((int64_t{1} << 31) - 1) / (8 * (ld > 0 ? ld : 1)) - 16;
  const int64_t min_ch = max_rows > 0 ? (M + max_rows - 1) / max_rows : M;
  if (ch < min_ch) ch = min_ch;
  if (ch < 1) ch = 1;
  return static_cast<int>(ch);
}

}  // namespace

size_t gram_partial_bytes(int64_t M, int n, int64_t ld) {
  const int npad = (n + kGT - 1) / kGT * kGT;
  return static_cast<size_t>(gram_chunks(M, n, ld)) * npad * npad * sizeof(double);
}

template <typename T>
hipError_t gram_t(const T* X, int64_t ldx, const T* Y, int64_t ldy, int64_t M, int n, double* partial,
                  double* G, int64_t ldg, hipStream_t s, int64_t offx, int64_t offy) {
  if (offx < 0 || offy < 0 || offx + n > ldx || offy + n > ldy) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  const int nt = (n + kGT - 1) / kGT;
  const int ntiles = nt * (nt + 1) / 2;
  const int npad = nt * kGT;
  int nch = gram_chunks(M, n, ldx > ldy ? ldx : ldy);
  int64_t rpc = (M + nch - 1) / nch;
  rpc = (rpc + 15) / 16 * 16;
  nch = static_cast<int>((M + rpc - 1) / rpc);   // rounding rpc up can leave trailing chunks empty
  hipLaunchKernelGGL((gram_kernel<T, kGramStages>), dim3(ntiles, nch), dim3(256), 0, s, X, ldx, Y, ldy, M, n, rpc,
                     npad, partial, offx, offy);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(blocks_for(static_cast<int64_t>(n) * n)), dim3(256), 0, s,
                     partial, nch, n, npad, G, ldg);
  return hipGetLastError();
}

hipError_t launch_gram(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t M, int n,
                       double* partial, double* G, int64_t ldg, hipStream_t s, int64_t offx, int64_t offy) {
  return gram_t(X, ldx, Y, ldy, M, n, partial, G, ldg, s, offx, offy);
}

hipError_t launch_gram(const float* X, int64_t ldx, const float* Y, int64_t ldy, int64_t M, int n,
                       double* partial, double* G, int64_t ldg, hipStream_t s, int64_t offx, int64_t offy) {
  return gram_t(X, ldx, Y, ldy, M, n, partial, G, ldg, s, offx, offy);
}

hipError_t launch_sym_from_lower(const double* G, int64_t ldg, double* S, int n, hipStream_t s) {
  hipLaunchKernelGGL(sym_from_lower_kernel, dim3(blocks_for(static_cast<int64_t>(n) * n)), dim3(256), 0, s,
                     G, ldg, S, n);
  return hipGetLastError();
}

hipError_t launch_gram_combine_complex(const double* G2, int64_t ldg2, double* S, int n, hipStream_t s) {
  hipLaunchKernelGGL(gram_combine_complex_kernel, dim3(blocks_for(static_cast<int64_t>(n) * n)), dim3(256), 0,
                     s, G2, ldg2, S, n);
  return hipGetLastError();
}

template <typename T>
hipError_t rotate_t(const T* X, int64_t ldx, const T* Z, int64_t ldz, T* C, int64_t ldc, int64_t M, int K, int N2,
                    bool upper, hipStream_t s) {
  if (M <= 0 || N2 <= 0) return hipSuccess;
  const int64_t gx = (M + kRM - 1) / kRM;
  if (gx > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rotate_kernel<T>, dim3(static_cast<unsigned>(gx), (N2 + kRN - 1) / kRN), dim3(256), 0, s, X,
                     ldx, Z, ldz, C, ldc, M, K, N2, upper ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_rotate(const double* X, int64_t ldx, const double* Z, int64_t ldz, double* C, int64_t ldc,
                         int64_t M, int K, int N2, bool upper, hipStream_t s) {
  return rotate_t(X, ldx, Z, ldz, C, ldc, M, K, N2, upper, s);
}

hipError_t launch_rotate(const float* X, int64_t ldx, const float* Z, int64_t ldz, float* C, int64_t ldc,
                         int64_t M, int K, int N2, bool upper, hipStream_t s) {
  return rotate_t(X, ldx, Z, ldz, C, ldc, M, K, N2, upper, s);
}

size_t resid_partial_count(int64_t M, int ncols) {
  (void)M;
  const int ny = (ncols + 255) / 256;
  int nch = 1024 / ny;
  if (nch < 1) nch = 1;
  return static_cast<size_t>(nch) * ncols;
}

hipError_t launch_resid(const double* HX, int64_t ldh, const double* X, int64_t ldx, const double* theta,
                        int64_t M, int ncols, bool cplx, double* partial, int* nchunks_out, hipStream_t s) {
  const int ny = (ncols + 255) / 256;
  int nch = 1024 / ny;
  if (nch < 1) nch = 1;
  const int64_t rpc = (M + nch - 1) / nch;
  *nchunks_out = nch;
  hipLaunchKernelGGL(resid_kernel, dim3(nch, ny), dim3(256), 0, s, HX, ldh, X, ldx, theta, M, ncols,
                     cplx ? 1 : 0, rpc, partial);
  return hipGetLastError();
}

int dot_blocks() { return kDotBlocks; }

hipError_t launch_dot(const double* x, const double* y, int64_t n, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(kDotBlocks), dim3(256), 0, s, x, y, n, partial);
  return hipGetLastError();
}

hipError_t launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(axpby_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, a, x, b, y, n);
  return hipGetLastError();
}

hipError_t launch_transpose_rect(const double* in, int64_t ldi, int rows, int cols, double* out, int64_t ldo,
                                 hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_rect_kernel, dim3(blocks_for(static_cast<int64_t>(rows) * cols)), dim3(256), 0, s,
                     in, ldi, rows, cols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_split_diag(const double* Z, int64_t ldz, int n, float* Zo, double* d, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_diag_kernel, dim3(blocks_for(static_cast<int64_t>(n) * n)), dim3(256), 0, s, Z, ldz, n,
                     Zo, d);
  return hipGetLastError();
}

hipError_t launch_add_scaled_cols(const float* C, int64_t ldc, const double* d, double* X, int64_t ldx, int64_t M,
                                  int n, hipStream_t s) {
  if (M <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_scaled_cols_kernel, dim3(blocks_for(M * n)), dim3(256), 0, s, C, ldc, d, X, ldx, M, n);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* in, double* out, int n, hipStream_t s) {
  hipLaunchKernelGGL(transpose_kernel, dim3(blocks_for(static_cast<int64_t>(n) * n)), dim3(256), 0, s, in, out,
                     n);
  return hipGetLastError();
}

hipError_t launch_zero_strict_lower(double* A, int n, int64_t lda, hipStream_t s) {
  hipLaunchKernelGGL(zero_strict_lower_kernel, dim3(blocks_for(static_cast<int64_t>(n) * n)), dim3(256), 0, s,
                     A, n, lda);
  return hipGetLastError();
}

hipError_t launch_expand_complex(const double* Z, int n1, int n2, int mode, double* Z2, hipStream_t s) {
  hipLaunchKernelGGL(expand_complex_kernel, dim3(blocks_for(static_cast<int64_t>(n1) * n2)), dim3(256), 0, s,
                     Z, n1, n2, mode, Z2);
  return hipGetLastError();
}

}  // namespace chfsi
