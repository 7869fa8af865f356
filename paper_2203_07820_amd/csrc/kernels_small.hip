// Dense kernels for small subspaces (N <= 64 columns) of the CholGS and
// Rayleigh-Ritz steps (Section 4.4, Algorithm 2): the Cholesky factor of the
// overlap S = L L^H with its inverse L^-1, and the Hermitian eigensolve of the
// projected Hamiltonian.  Each matrix is handled by one workgroup with the
// whole matrix in LDS, and a launch covers any number of matrices (one
// workgroup each), so a batch of small problems needs one launch per step.
// For small N the solver library's routines are bound by their own launches
// and host synchronisations, not by arithmetic; these kernels report failure
// through a device flag that the host reads with the pass's results.
//
// Layout: every matrix is column-major, n x n, element (i, j) at i + j n
// (complex: interleaved re, im), as the library routines they stand in for.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "internal.h"

namespace chfsi {
namespace {

constexpr int kSmallThreads = 256;

struct cd {
  double re, im;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cmulc(cd a, cd b) { return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im}; }  // a conj(b)

// Element access for real (CPLX = false: im ignored, kept 0) and complex data,
// in LDS or (through a gptr) in global memory.
template <bool CPLX, typename Ptr> __device__ __forceinline__ cd ld_el(Ptr m, int64_t e) {
  if constexpr (CPLX) return {m[2 * e], m[2 * e + 1]};
  else return {m[e], 0.0};
}
template <bool CPLX, typename Ptr> __device__ __forceinline__ void st_el(Ptr m, int64_t e, cd v) {
  if constexpr (CPLX) {
    m[2 * e] = v.re;
    m[2 * e + 1] = v.im;
  } else {
    m[e] = v.re;
  }
}

// ---- Cholesky factor and its inverse ---------------------------------------
// S (lower triangle read) -> lower triangle of S overwritten with L^-1, where
// S = L L^H.  info = 0, or k + 1 if the k-th pivot is not positive to
// working precision, i.e. not above 16 eps S_kk: column k is then a linear
// combination of the earlier ones up to rounding (a block whose condition
// number exceeds about 1/sqrt(16 eps), where Cholesky orthonormalisation
// loses all orthogonality anyway); the factorisation stops there and S is
// left as it was.
// Right-looking factorisation in LDS (L row-major with a padded row), then
// forward substitution with one column of L^-1 per thread (no barriers),
// the column built in LDS: each entry depends on the column's earlier ones,
// which read back from global memory would put an L2 round trip on every
// step of the chain.
template <bool CPLX>
__global__ void __launch_bounds__(kSmallThreads)
small_cholinv_kernel(const SmallBatch b) {
  constexpr int CF = CPLX ? 2 : 1;
  __shared__ double sm[kSmallMaxN * (kSmallMaxN + 1) * CF + 2 * kSmallMaxN];
  __shared__ double xs[kSmallMaxN * kSmallMaxN * CF];   // L^-1, X[i][j] at (i kSmallMaxN + j) CF
  const gptr<double> S = to_global(b.mats ? b.mats[blockIdx.x] : b.mat0);
  const int n = b.dims ? b.dims[blockIdx.x] : b.n0;
  const gptr<int> info = to_global(b.info);
  const int ld = n + 1;
  double* L = sm;                        // L[i][j] at (i ld + j) CF, j <= i
  double* dg = sm + static_cast<int64_t>(n) * ld * CF;   // diagonal of L
  double* s0 = dg + n;                                    // diagonal of S
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kSmallThreads) {
    const int i = e % n, j = e / n;
    if (i >= j) st_el<CPLX>(L, static_cast<int64_t>(i) * ld + j, ld_el<CPLX>(S, e));
    if (i == j) s0[i] = S[e * CF];
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double d = L[(static_cast<int64_t>(k) * ld + k) * CF];   // real part (Hermitian diagonal)
    // uniform: every thread read the same d and s0[k]
    if (!(d > 16.0 * __DBL_EPSILON__ * s0[k]) || !(d > 0.0) || !(d < INFINITY)) {
      if (tid == 0) info[blockIdx.x] = k + 1;
      return;
    }
    const double lkk = sqrt(d), inv = 1.0 / lkk;
    if (tid == 0) dg[k] = lkk;
    for (int i = k + 1 + tid; i < n; i += kSmallThreads) {
      const int64_t e = static_cast<int64_t>(i) * ld + k;
      cd v = ld_el<CPLX>(L, e);
      st_el<CPLX>(L, e, {v.re * inv, v.im * inv});
    }
    __syncthreads();
    // trailing update of the lower triangle: L[i][j] -= L[i][k] conj(L[j][k])
    const int nt = n - 1 - k;
    for (int e = tid; e < nt * nt; e += kSmallThreads) {
      const int i = k + 1 + e / nt, j = k + 1 + e % nt;
      if (j > i) continue;
      const cd lik = ld_el<CPLX>(L, static_cast<int64_t>(i) * ld + k);
      const cd ljk = ld_el<CPLX>(L, static_cast<int64_t>(j) * ld + k);
      const int64_t o = static_cast<int64_t>(i) * ld + j;
      const cd a = ld_el<CPLX>(L, o), pr = cmulc(lik, ljk);
      st_el<CPLX>(L, o, {a.re - pr.re, a.im - pr.im});
    }
    __syncthreads();
  }
  // X = L^-1 (lower): column j by thread j, X[i][j] = (delta_ij - sum_{k=j}^{i-1} L[i][k] X[k][j]) / L[i][i],
  // kept in xs (column j of X only depends on itself) and stored into S's
  // lower triangle, whose column j is no longer read
  for (int j = tid; j < n; j += kSmallThreads) {
    for (int i = j; i < n; ++i) {
      cd s = {i == j ? 1.0 : 0.0, 0.0};
      for (int k = j; k < i; ++k) {
        const cd p = cmul(ld_el<CPLX>(L, static_cast<int64_t>(i) * ld + k),
                          ld_el<CPLX>(xs, static_cast<int64_t>(k) * kSmallMaxN + j));
        s.re -= p.re;
        s.im -= p.im;
      }
      const double r = 1.0 / dg[i];
      const cd x = {s.re * r, s.im * r};
      st_el<CPLX>(xs, static_cast<int64_t>(i) * kSmallMaxN + j, x);
      st_el<CPLX>(S, i + static_cast<int64_t>(j) * n, x);
    }
  }
  if (tid == 0) info[blockIdx.x] = 0;
}

// ---- Hermitian eigensolve --------------------------------------------------
// H (lower triangle read) -> H overwritten with the eigenvectors (column j for
// the j-th eigenvalue), D = eigenvalues in ascending order; info = 0, or 1 if
// the iteration did not converge.  Cyclic Jacobi with the round-robin order:
// each of the m - 1 rounds of a sweep (m = n rounded up to even) rotates m / 2
// disjoint index pairs at once.  For a pair (p, q) with a_pq = r w (r = |a_pq|,
// |w| = 1), U = diag(1, conj(w)) R, R = [[c, s], [-s, c]] the real rotation
// that diagonalises [[a_pp, r], [r, a_qq]]; A <- U^H A U is applied by 2 x 2
// blocks (all rotations of a round act on disjoint index pairs, so each block
// sees exactly its row pair's and column pair's rotations), V <- V U beside
// it: two barriers per round.  A sweep starts only while the off-diagonal
// mass exceeds 1e-30 of the total.
template <bool CPLX>
__global__ void __launch_bounds__(kSmallThreads)
small_eigh_kernel(const SmallBatch b) {
  constexpr int CF = CPLX ? 2 : 1;
  constexpr int kMaxSweeps = 50;
  __shared__ double sm[2 * kSmallMaxN * (kSmallMaxN + 1) * CF + 4 * (kSmallMaxN / 2)];
  __shared__ int pq[kSmallMaxN];          // per pair: p, q (an index >= n: the dummy of odd n)
  __shared__ int actf[kSmallMaxN / 2];    // per pair: 1 if rotated this round
  const gptr<double> H = to_global(b.mats ? b.mats[blockIdx.x] : b.mat0);
  const int n = b.dims ? b.dims[blockIdx.x] : b.n0;
  const gptr<double> D = to_global(b.evals ? b.evals[blockIdx.x] : b.ev0);
  const gptr<int> info = to_global(b.info);
  const int ld = n + 1;
  const int m = n + (n & 1);
  const int np = m / 2;
  double* A = sm;                                        // A[i][j] at (i ld + j) CF
  double* V = sm + static_cast<int64_t>(n) * ld * CF;    // V[i][j] likewise
  double* rot = V + static_cast<int64_t>(n) * ld * CF;   // per pair: c, s, w.re, w.im
  __shared__ double red[2 * kSmallThreads];
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kSmallThreads) {
    const int i = e % n, j = e / n;
    const int64_t o = static_cast<int64_t>(i) * ld + j;
    if (i >= j) {
      cd v = ld_el<CPLX>(H, e);
      if (i == j) v.im = 0.0;
      st_el<CPLX>(A, o, v);
      st_el<CPLX>(A, static_cast<int64_t>(j) * ld + i, {v.re, -v.im});
    }
    st_el<CPLX>(V, o, {i == j ? 1.0 : 0.0, 0.0});
  }
  __syncthreads();
  bool converged = n <= 1;
  for (int sweep = 0; sweep < kMaxSweeps && !converged; ++sweep) {
    // off-diagonal and total mass
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += kSmallThreads) {
      const int i = e / n, j = e % n;
      const cd v = ld_el<CPLX>(A, static_cast<int64_t>(i) * ld + j);
      const double a2 = v.re * v.re + v.im * v.im;
      tot += a2;
      if (i != j) off += a2;
    }
    red[tid] = off;
    red[kSmallThreads + tid] = tot;
    __syncthreads();
    for (int w = kSmallThreads / 2; w > 0; w >>= 1) {
      if (tid < w) {
        red[tid] += red[tid + w];
        red[kSmallThreads + tid] += red[kSmallThreads + tid + w];
      }
      __syncthreads();
    }
    converged = red[0] <= 1e-30 * red[kSmallThreads];
    __syncthreads();   // red is rewritten by the next sweep
    if (converged) break;
    for (int r = 0; r < m - 1; ++r) {
      // 1. rotation of every pair of this round
      if (tid < np) {
        int p, q;
        if (tid == 0) {
          p = r;
          q = m - 1;
        } else {
          p = (r + tid) % (m - 1);
          q = (r - tid + m - 1) % (m - 1);
        }
        double c = 1.0, s = 0.0, wr = 1.0, wi = 0.0;
        bool act = p < n && q < n;
        if (act) {
          const cd apq = ld_el<CPLX>(A, static_cast<int64_t>(p) * ld + q);
          double rr = CPLX ? sqrt(apq.re * apq.re + apq.im * apq.im) : apq.re;
          if (fabs(rr) <= 1e-300) {
            act = false;
          } else {
            if constexpr (CPLX) {
              wr = apq.re / rr;
              wi = apq.im / rr;
            }
            const double app = A[(static_cast<int64_t>(p) * ld + p) * CF];
            const double aqq = A[(static_cast<int64_t>(q) * ld + q) * CF];
            const double th = (aqq - app) / (2.0 * rr);
            const double t = fabs(th) < 1e150 ? (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0))
                                              : 0.5 / th;
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        rot[4 * tid] = c;
        rot[4 * tid + 1] = s;
        rot[4 * tid + 2] = wr;
        rot[4 * tid + 3] = wi;
        pq[2 * tid] = p;
        pq[2 * tid + 1] = q;
        actf[tid] = act ? 1 : 0;
      }
      __syncthreads();
      // 2. A <- U^H A U by 2 x 2 blocks (rows of pair k, columns of pair l):
      //    rows p' = c A_p - s w A_q, q' = s A_p + c w A_q, then columns
      //    p' = c A_p - s conj(w) A_q, q' = s A_p + c conj(w) A_q; disjoint
      //    blocks, so one phase; a rotated pair's own off-diagonal entries
      //    are set to exactly zero.  V <- V U in the same phase.
      for (int b = tid; b < np * np; b += kSmallThreads) {
        const int k = b / np, l = b % np;
        if (!actf[k] && !actf[l]) continue;
        const int i0 = pq[2 * k], i1 = pq[2 * k + 1], j0 = pq[2 * l], j1 = pq[2 * l + 1];
        const bool r0 = i0 < n, r1 = i1 < n, c0 = j0 < n, c1 = j1 < n;
        const int64_t o00 = static_cast<int64_t>(i0) * ld + j0, o01 = static_cast<int64_t>(i0) * ld + j1;
        const int64_t o10 = static_cast<int64_t>(i1) * ld + j0, o11 = static_cast<int64_t>(i1) * ld + j1;
        const cd zero = {0.0, 0.0};
        cd b00 = (r0 && c0) ? ld_el<CPLX>(A, o00) : zero, b01 = (r0 && c1) ? ld_el<CPLX>(A, o01) : zero;
        cd b10 = (r1 && c0) ? ld_el<CPLX>(A, o10) : zero, b11 = (r1 && c1) ? ld_el<CPLX>(A, o11) : zero;
        if (actf[k]) {
          const double c = rot[4 * k], s = rot[4 * k + 1];
          const cd w = {rot[4 * k + 2], rot[4 * k + 3]};
          const cd w10 = CPLX ? cmul(w, b10) : b10, w11 = CPLX ? cmul(w, b11) : b11;
          const cd n00 = {c * b00.re - s * w10.re, c * b00.im - s * w10.im};
          const cd n01 = {c * b01.re - s * w11.re, c * b01.im - s * w11.im};
          const cd n10 = {s * b00.re + c * w10.re, s * b00.im + c * w10.im};
          const cd n11 = {s * b01.re + c * w11.re, s * b01.im + c * w11.im};
          b00 = n00; b01 = n01; b10 = n10; b11 = n11;
        }
        if (actf[l]) {
          const double c = rot[4 * l], s = rot[4 * l + 1];
          const cd wc = {rot[4 * l + 2], -rot[4 * l + 3]};
          const cd w01 = CPLX ? cmul(wc, b01) : b01, w11 = CPLX ? cmul(wc, b11) : b11;
          const cd n00 = {c * b00.re - s * w01.re, c * b00.im - s * w01.im};
          const cd n10 = {c * b10.re - s * w11.re, c * b10.im - s * w11.im};
          const cd n01 = {s * b00.re + c * w01.re, s * b00.im + c * w01.im};
          const cd n11 = {s * b10.re + c * w11.re, s * b10.im + c * w11.im};
          b00 = n00; b01 = n01; b10 = n10; b11 = n11;
        }
        if (k == l) {   // the rotated pair: its off-diagonal entries vanish
          b01 = zero;
          b10 = zero;
        }
        if (r0 && c0) st_el<CPLX>(A, o00, b00);
        if (r0 && c1) st_el<CPLX>(A, o01, b01);
        if (r1 && c0) st_el<CPLX>(A, o10, b10);
        if (r1 && c1) st_el<CPLX>(A, o11, b11);
      }
      for (int e = tid; e < n * np; e += kSmallThreads) {
        const int i = e / np, l = e % np;
        if (!actf[l]) continue;
        const int j0 = pq[2 * l], j1 = pq[2 * l + 1];   // both < n for a rotated pair
        const double c = rot[4 * l], s = rot[4 * l + 1];
        const cd wc = {rot[4 * l + 2], -rot[4 * l + 3]};
        const int64_t o0 = static_cast<int64_t>(i) * ld + j0, o1 = static_cast<int64_t>(i) * ld + j1;
        const cd v0 = ld_el<CPLX>(V, o0), v1 = ld_el<CPLX>(V, o1);
        const cd wv1 = CPLX ? cmul(wc, v1) : v1;
        st_el<CPLX>(V, o0, {c * v0.re - s * wv1.re, c * v0.im - s * wv1.im});
        st_el<CPLX>(V, o1, {s * v0.re + c * wv1.re, s * v0.im + c * wv1.im});
      }
      __syncthreads();
    }
  }
  // eigenvalues in ascending order (ties by index), vectors to the same columns
  for (int i = tid; i < n; i += kSmallThreads) {
    const double di = A[(static_cast<int64_t>(i) * ld + i) * CF];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = A[(static_cast<int64_t>(j) * ld + j) * CF];
      rank += (dj < di || (dj == di && j < i)) ? 1 : 0;
    }
    D[rank] = di;
    for (int row = 0; row < n; ++row)
      st_el<CPLX>(H, row + static_cast<int64_t>(rank) * n, ld_el<CPLX>(V, static_cast<int64_t>(row) * ld + i));
  }
  if (tid == 0) info[blockIdx.x] = converged ? 0 : 1;
}

}  // namespace

hipError_t launch_small_cholinv(const SmallBatch& b, int count, bool cplx, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (cplx) hipLaunchKernelGGL(small_cholinv_kernel<true>, dim3(count), dim3(kSmallThreads), 0, s, b);
  else hipLaunchKernelGGL(small_cholinv_kernel<false>, dim3(count), dim3(kSmallThreads), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_small_eigh(const SmallBatch& b, int count, bool cplx, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (cplx) hipLaunchKernelGGL(small_eigh_kernel<true>, dim3(count), dim3(kSmallThreads), 0, s, b);
  else hipLaunchKernelGGL(small_eigh_kernel<false>, dim3(count), dim3(kSmallThreads), 0, s, b);
  return hipGetLastError();
}

}  // namespace chfsi
