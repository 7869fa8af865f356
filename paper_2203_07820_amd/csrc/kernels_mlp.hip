// Kernels of the learned warm start: per-node radial features of the atoms,
// a 3-layer tanh MLP (forward and backward) on FP32 MFMA, the rotation- and
// sign-invariant subspace loss and Adam.  All contractions are tall-skinny:
// rows are nodes (M ~ 10^5..10^6), columns are at most 128.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace chfsi {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register i holds D[4 (l / 16) + i][l % 16].
__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---- C = epi(A W): A (M x K, lda), W (K x N) with strides (swk, swn) -------
constexpr int kGM = 64, kGN = 128, kGK = 16;

__global__ void __launch_bounds__(256)
mlp_gemm_kernel(const float* __restrict__ A, int64_t lda, const float* __restrict__ W, int64_t swk, int64_t swn,
                float* __restrict__ C, int64_t ldc, int64_t M, int K, int N, int mode, const float* __restrict__ bias,
                const float* __restrict__ D0, int64_t ldd) {
  __shared__ float as[kGM][kGK + 1];
  __shared__ float ws[kGK][kGN];
  const int64_t r0 = blockIdx.x * static_cast<int64_t>(kGM);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  f4 acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = f4{0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < kGM * kGK / 256; ++i) {
      const int e = tid + 256 * i;
      const int r = e / kGK, k = e % kGK;
      const int64_t row = r0 + r;
      as[r][k] = (row < M && k0 + k < K) ? A[row * lda + k0 + k] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < kGK * kGN / 256; ++i) {
      const int e = tid + 256 * i;
      const int k = e / kGN, n = e % kGN;
      ws[k][n] = (k0 + k < K && n < N) ? W[(k0 + k) * swk + n * swn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      const float av = as[wave * 16 + lane % 16][ks * 4 + lane / 16];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = mma(av, ws[ks * 4 + lane / 16][q * 16 + lane % 16], acc[q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = r0 + wave * 16 + 4 * (lane / 16) + i;
      const int col = q * 16 + lane % 16;
      if (row >= M || col >= N) continue;
      float v = acc[q][i];
      if (bias) v += bias[col];
      if (mode == 1) {
        v = tanhf(v);
      } else if (mode == 2) {
        v = D0[row * ldd + col] - v;
      } else if (mode == 3) {
        const float t = D0[row * ldd + col];
        v = v * (1.f - t * t);
      }
      C[row * ldc + col] = v;
    }
}

// ---- partial[chunk] = A^T B over the chunk's rows (KA, KB <= 128) ---------
constexpr int kTT = 128, kTK = 16;

__global__ void __launch_bounds__(256)
mlp_gram_kernel(const float* __restrict__ A, int64_t lda, int KA, const float* __restrict__ B, int64_t ldb,
                int KB, int64_t M, int64_t rows_per_chunk, float* __restrict__ part) {
  __shared__ float xs[kTK][kTT];
  __shared__ float ys[kTK][kTT];
  const int chunk = blockIdx.x;
  const int64_t m0 = chunk * rows_per_chunk;
  int64_t m1 = m0 + rows_per_chunk;
  if (m1 > M) m1 = M;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wi = (wave / 2) * 64, wj = (wave % 2) * 64;
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};
  const int lc = tid % kTT, lr = tid / kTT;
  for (int64_t m = m0; m < m1; m += kTK) {
#pragma unroll
    for (int i = 0; i < kTK / 2; ++i) {
      const int r = lr + 2 * i;
      const int64_t row = m + r;
      xs[r][lc] = (row < m1 && lc < KA) ? A[row * lda + lc] : 0.f;
      ys[r][lc] = (row < m1 && lc < KB) ? B[row * ldb + lc] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kTK / 4; ++ks) {
      const int kr = ks * 4 + lane / 16;
      float av[4], bv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        av[q] = xs[kr][wi + q * 16 + lane % 16];
        bv[q] = ys[kr][wj + q * 16 + lane % 16];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  float* out = part + static_cast<int64_t>(chunk) * kTT * kTT;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out[(wi + a * 16 + 4 * (lane / 16) + i) * kTT + wj + b * 16 + lane % 16] = acc[a][b][i];
}

// G[i][j] (KA x KB, ldg) = sum over chunks, summed in FP64 in fixed order.
__global__ void mlp_gram_reduce_kernel(const float* __restrict__ part, int nchunks, int KA, int KB,
                                       float* __restrict__ G, int ldg) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= KA * KB) return;
  const int i = idx / KB, j = idx % KB;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(static_cast<int64_t>(c) * kTT + i) * kTT + j];
  G[i * ldg + j] = static_cast<float>(s);
}

// column sums: partial[chunk][j] over the chunk's rows
__global__ void mlp_colsum_kernel(const float* __restrict__ A, int64_t lda, int N, int64_t M,
                                  int64_t rows_per_chunk, double* __restrict__ part) {
  const int j = threadIdx.x;
  if (j >= N) return;
  const int64_t m0 = blockIdx.x * rows_per_chunk;
  int64_t m1 = m0 + rows_per_chunk;
  if (m1 > M) m1 = M;
  double s = 0.0;
  for (int64_t r = m0; r < m1; ++r) s += A[r * lda + j];
  part[static_cast<int64_t>(blockIdx.x) * N + j] = s;
}

__global__ void mlp_colsum_reduce_kernel(const double* __restrict__ part, int nchunks, int N, float* out) {
  const int j = threadIdx.x;
  if (j >= N) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[static_cast<int64_t>(c) * N + j];
  out[j] = static_cast<float>(s);
}

// partial sums of x.y over a row-major M x N block (contiguous, ld = N)
__global__ void __launch_bounds__(256)
mlp_dot_kernel(const float* __restrict__ x, const float* __restrict__ y, int64_t n, double* part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * 256)
    s += static_cast<double>(x[i]) * y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// D = (n / s) G - I for the n x n Gram G = Y^T Y; out[0] = sum D .* G,
// out[1] = sum D .* D (one workgroup, FP64 accumulation).
__global__ void __launch_bounds__(256)
mlp_loss_small_kernel(const float* __restrict__ G, int n, double s, float* __restrict__ D, double* out) {
  __shared__ double r0[256], r1[256];
  double a = 0.0, b = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += 256) {
    const int i = idx / n, j = idx % n;
    const double g = G[idx];
    const double d = (n / s) * g - (i == j ? 1.0 : 0.0);
    D[idx] = static_cast<float>(d);
    a += d * g;
    b += d * d;
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
  }
}

// dY = c1 R + c2 Y + c3 YD (contiguous M x N blocks)
__global__ void mlp_combine_kernel(float c1, const float* __restrict__ R, float c2, const float* __restrict__ Y,
                                   float c3, const float* __restrict__ YD, float* __restrict__ dY, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dY[i] = c1 * R[i] + c2 * Y[i] + c3 * YD[i];
}

__global__ void mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                                float c2) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Fn = (F - mean) / std, M x din contiguous
__global__ void mlp_normalize_kernel(const float* __restrict__ F, const float* __restrict__ mean,
                                     const float* __restrict__ stdv, float* __restrict__ Fn, int64_t M, int din) {
  const int64_t total = M * din;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int k = static_cast<int>(i % din);
    Fn[i] = (F[i] - mean[k]) / stdv[k];
  }
}

// Radial features: F[j][8 q + k] = sum_a sum_images phi_q(a) exp(-(r - k)^2 / (2 eta^2)),
// r = |x_j - R_a - nL| <= rcut; atoms[a] = (x, y, z, Z, s, h_s, h_p, -).
__global__ void __launch_bounds__(256)
features_kernel(const double* __restrict__ x1d, int n, double L, const double* __restrict__ atoms, int natoms,
                int kimg, double eta, double rcut, float* __restrict__ F) {
  const int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t M = static_cast<int64_t>(n) * n * n;
  if (j >= M) return;
  const double x = x1d[j % n], y = x1d[(j / n) % n], z = x1d[j / (static_cast<int64_t>(n) * n)];
  double acc[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) acc[i] = 0.0;
  const double inv = 1.0 / (2.0 * eta * eta);
  for (int a = 0; a < natoms; ++a) {
    const double* at = atoms + 8 * a;
    for (int iz = -kimg; iz <= kimg; ++iz)
      for (int iy = -kimg; iy <= kimg; ++iy)
        for (int ix = -kimg; ix <= kimg; ++ix) {
          const double dx = x - (at[0] + ix * L), dy = y - (at[1] + iy * L), dz = z - (at[2] + iz * L);
          const double r = sqrt(dx * dx + dy * dy + dz * dz);
          if (r > rcut) continue;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const double g = exp(-(r - k) * (r - k) * inv);
            acc[k] += at[3] * g;
            acc[8 + k] += at[4] * g;
            acc[16 + k] += at[5] * g;
            acc[24 + k] += at[6] * g;
          }
        }
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) F[j * 32 + i] = static_cast<float>(acc[i]);
}

unsigned grid1(int64_t n, int per = 256, int64_t cap = 8192) {
  int64_t g = (n + per - 1) / per;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return static_cast<unsigned>(g);
}

}  // namespace

hipError_t mlp_gemm(const float* A, int64_t lda, const float* W, int64_t swk, int64_t swn, float* C, int64_t ldc,
                    int64_t M, int K, int N, int mode, const float* bias, const float* D0, int64_t ldd, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (N > kGN || K <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_gemm_kernel, dim3(static_cast<unsigned>((M + kGM - 1) / kGM)), dim3(256), 0, s, A, lda, W,
                     swk, swn, C, ldc, M, K, N, mode, bias, D0, ldd);
  return hipGetLastError();
}

int mlp_gram_chunks(int64_t M) {
  int64_t c = (M + 2047) / 2048;
  if (c > 512) c = 512;
  if (c < 1) c = 1;
  return static_cast<int>(c);
}

size_t mlp_gram_partial_bytes(int64_t M) { return static_cast<size_t>(mlp_gram_chunks(M)) * kTT * kTT * 4; }

hipError_t mlp_gram(const float* A, int64_t lda, int KA, const float* B, int64_t ldb, int KB, int64_t M, float* part,
                    float* G, int ldg, hipStream_t s) {
  if (KA > kTT || KB > kTT) return hipErrorInvalidValue;
  const int nch = mlp_gram_chunks(M);
  int64_t rpc = (M + nch - 1) / nch;
  rpc = (rpc + kTK - 1) / kTK * kTK;
  hipLaunchKernelGGL(mlp_gram_kernel, dim3(nch), dim3(256), 0, s, A, lda, KA, B, ldb, KB, M, rpc, part);
  hipLaunchKernelGGL(mlp_gram_reduce_kernel, dim3((KA * KB + 255) / 256), dim3(256), 0, s, part, nch, KA, KB, G, ldg);
  return hipGetLastError();
}

size_t mlp_colsum_partial_bytes(int64_t M, int N) { return static_cast<size_t>(mlp_gram_chunks(M)) * N * 8; }

hipError_t mlp_colsum(const float* A, int64_t lda, int N, int64_t M, double* part, float* out, hipStream_t s) {
  if (N > 256) return hipErrorInvalidValue;
  const int nch = mlp_gram_chunks(M);
  const int64_t rpc = (M + nch - 1) / nch;
  hipLaunchKernelGGL(mlp_colsum_kernel, dim3(nch), dim3(256), 0, s, A, lda, N, M, rpc, part);
  hipLaunchKernelGGL(mlp_colsum_reduce_kernel, dim3(1), dim3(256), 0, s, part, nch, N, out);
  return hipGetLastError();
}

int mlp_dot_blocks() { return 512; }

hipError_t mlp_dot(const float* x, const float* y, int64_t n, double* part, hipStream_t s) {
  hipLaunchKernelGGL(mlp_dot_kernel, dim3(512), dim3(256), 0, s, x, y, n, part);
  return hipGetLastError();
}

hipError_t mlp_loss_small(const float* G, int n, double sY, float* D, double* out, hipStream_t s) {
  hipLaunchKernelGGL(mlp_loss_small_kernel, dim3(1), dim3(256), 0, s, G, n, sY, D, out);
  return hipGetLastError();
}

hipError_t mlp_combine(float c1, const float* R, float c2, const float* Y, float c3, const float* YD, float* dY,
                       int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(mlp_combine_kernel, dim3(grid1(n)), dim3(256), 0, s, c1, R, c2, Y, c3, YD, dY, n);
  return hipGetLastError();
}

hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                    int t, hipStream_t s) {
  const float c1 = 1.f - powf(b1, static_cast<float>(t));
  const float c2 = 1.f - powf(b2, static_cast<float>(t));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(grid1(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_normalize(const float* F, const float* mean, const float* stdv, float* Fn, int64_t M, int din,
                         hipStream_t s) {
  hipLaunchKernelGGL(mlp_normalize_kernel, dim3(grid1(M * din)), dim3(256), 0, s, F, mean, stdv, Fn, M, din);
  return hipGetLastError();
}

hipError_t launch_features(const double* x1d, int n, double L, const double* atoms, int natoms, int kimg, double eta,
                           double rcut, float* F, hipStream_t s) {
  const int64_t M = static_cast<int64_t>(n) * n * n;
  hipLaunchKernelGGL(features_kernel, dim3(static_cast<unsigned>((M + 255) / 256)), dim3(256), 0, s, x1d, n, L, atoms,
                     natoms, kimg, eta, rcut, F);
  return hipGetLastError();
}

}  // namespace chfsi
