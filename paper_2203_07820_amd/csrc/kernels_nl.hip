// Node-level projector contraction of the nonlocal Hamiltonian (DFT-FE 1.0,
// Eq. nonlocalHamDiscrete and Algorithm 4, the steps that form the
// projections P_a = h_a sum_j conj(c~_{a,j}) X_j), and the elementwise
// helpers of the filter (zero fill, precision conversion of a block).
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "internal.h"

namespace chfsi {
namespace {

// ---- node-level projector contraction (Algorithm 4 steps 1-4) -------------
// P_a = h_a * sum_j conj(c~_{a,j}) X[j, :], computed from atom-major node
// lists (each node row read once per atom), in two deterministic phases:
// fixed-size chunks of an atom's list give partial sums, then the chunks of
// each atom are summed in order and scaled by the couplings.
constexpr int kNlChunk = 512;

// One workgroup: one chunk of an atom's node list and 64 columns; wave w
// takes the entries w, w + 4, ...  Entries go in groups of 8 per wave: their
// node ids and projector values are wave-uniform (scalar loads), the 8 row
// loads of X are issued before any is used, so their latencies overlap.
template <typename T, bool CPLX>
__device__ __forceinline__ void nl_partial_item(const int chunk, const int ctile, gptr<const int32_t> chunk_atom,
                                                gptr<const int64_t> chunk_begin, gptr<const int64_t> atom_ptr,
                                                gptr<const int32_t> atom_node, gptr<const double> atom_val,
                                                gptr<const T> X, int64_t ldx, int ncols, gptr<T> partial,
                                                int64_t ldhp) {
  __shared__ T red[4][CPLX ? 8 : 4][64];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  const int col = ctile * 64 + lane;  // logical column
  const int colc = col < ncols ? col : ncols - 1;
  const int at = chunk_atom[chunk];
  const int64_t e0 = chunk_begin[chunk];
  int64_t e1 = e0 + kNlChunk;
  if (e1 > atom_ptr[at + 1]) e1 = atom_ptr[at + 1];
  constexpr int NV = CPLX ? 8 : 4;
  constexpr int G = 8;
  T acc[NV];
#pragma unroll
  for (int m = 0; m < NV; ++m) acc[m] = T(0);
  auto add = [&](int64_t e, T xr, T xi) {
    const gptr<const double> v = atom_val + e * NV;
    if constexpr (CPLX) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const T cr = static_cast<T>(v[2 * m]), ci = static_cast<T>(v[2 * m + 1]);
        acc[2 * m] += cr * xr + ci * xi;       // conj(c) x, real part
        acc[2 * m + 1] += cr * xi - ci * xr;   // imaginary part
      }
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] += static_cast<T>(v[m]) * xr;
    }
  };
  int64_t e = e0 + wave;
  for (; e + 4 * (G - 1) < e1; e += 4 * G) {
    T xr[G], xi[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t j = atom_node[e + 4 * g];
      if constexpr (CPLX) {
        xr[g] = X[(j * ldx + colc) * 2];
        xi[g] = X[(j * ldx + colc) * 2 + 1];
      } else {
        xr[g] = X[j * ldx + colc];
        xi[g] = T(0);
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) add(e + 4 * g, xr[g], xi[g]);
  }
  for (; e < e1; e += 4) {
    const int64_t j = atom_node[e];
    if constexpr (CPLX)
      add(e, X[(j * ldx + colc) * 2], X[(j * ldx + colc) * 2 + 1]);
    else
      add(e, X[j * ldx + colc], T(0));
  }
#pragma unroll
  for (int m = 0; m < NV; ++m) red[wave][m][lane] = acc[m];
  __syncthreads();
  if (wave == 0 && col < ncols) {
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const T s = ((red[0][m][lane] + red[1][m][lane]) + red[2][m][lane]) + red[3][m][lane];
      if constexpr (CPLX) {
        partial[(static_cast<int64_t>(chunk) * 4 + m / 2) * ldhp + 2 * col + (m & 1)] = s;
      } else {
        partial[(static_cast<int64_t>(chunk) * 4 + m) * ldhp + col] = s;
      }
    }
  }
}

template <typename T, bool CPLX>
__global__ void __launch_bounds__(256)
nl_partial_kernel(const int32_t* chunk_atom, const int64_t* chunk_begin, const int64_t* atom_ptr,
                  const int32_t* atom_node, const double* atom_val, const T* X, int64_t ldx,
                  int ncols, T* partial, int64_t ldhp) {
  nl_partial_item<T, CPLX>(blockIdx.x, blockIdx.y, to_global(chunk_atom), to_global(chunk_begin),
                           to_global(atom_ptr), to_global(atom_node), to_global(atom_val), to_global(X), ldx, ncols,
                           to_global(partial), ldhp);
}

template <typename T>
__device__ __forceinline__ void nl_reduce_item(const int am, const int jblk, gptr<const int32_t> atom_chunk_ptr,
                                               gptr<const double> hcoef, gptr<const T> partial, gptr<T> hP,
                                               int64_t ldhp, int nreal) {
  const int at = am / 4, m = am % 4;   // am = atom * 4 + component
  const int j = jblk * 256 + threadIdx.x;
  if (j >= ldhp) return;
  T s = T(0);
  if (j < nreal) {
    for (int ch = atom_chunk_ptr[at]; ch < atom_chunk_ptr[at + 1]; ++ch)
      s += partial[(static_cast<int64_t>(ch) * 4 + m) * ldhp + j];
    s *= static_cast<T>(hcoef[am]);
  }
  hP[static_cast<int64_t>(am) * ldhp + j] = s;
}

template <typename T>
__global__ void __launch_bounds__(256)
nl_reduce_kernel(const int32_t* atom_chunk_ptr, const double* hcoef, const T* partial, T* hP,
                 int64_t ldhp, int nreal) {
  nl_reduce_item<T>(blockIdx.x, blockIdx.y, to_global(atom_chunk_ptr), to_global(hcoef), to_global(partial),
                    to_global(hP), ldhp, nreal);
}

// The projection of many operators' blocks in two launches: work units are
// the concatenated chunks (partial sums) and (atom, component) rows (the
// reduction) of every problem; per-problem tables and pointers come from the
// device descriptors d[q].
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256)
nl_partial_batched_kernel(const NlLaunch* __restrict__ d, const int64_t* __restrict__ chunk_off, const int nprob) {
  const int q = problem_of(chunk_off, nprob, blockIdx.x);
  const NlLaunch& L = d[q];
  if (static_cast<int>(blockIdx.y) * 64 >= L.ncols) return;
  nl_partial_item<T, CPLX>(static_cast<int>(blockIdx.x - chunk_off[q]), blockIdx.y, to_global(L.chunk_atom),
                           to_global(L.chunk_begin), to_global(L.atom_ptr), to_global(L.atom_node),
                           to_global(L.atom_val), to_global(static_cast<const T*>(L.X)), L.ldx, L.ncols,
                           to_global(static_cast<T*>(L.partial)), L.ldhp);
}

template <typename T, bool CPLX>
__global__ void __launch_bounds__(256)
nl_reduce_batched_kernel(const NlLaunch* __restrict__ d, const int64_t* __restrict__ am_off, const int nprob) {
  const int q = problem_of(am_off, nprob, blockIdx.x);
  const NlLaunch& L = d[q];
  nl_reduce_item<T>(static_cast<int>(blockIdx.x - am_off[q]), blockIdx.y, to_global(L.atom_chunk_ptr),
                    to_global(L.hcoef), to_global(static_cast<const T*>(L.partial)),
                    to_global(static_cast<T*>(L.hP)), L.ldhp, CPLX ? 2 * L.ncols : L.ncols);
}

template <typename T, bool CPLX>
hipError_t nl_launch(const NlLaunch& L, hipStream_t s) {
  if (L.nchunks <= 0) return hipSuccess;
  const int nct = (L.ncols + 63) / 64;
  hipLaunchKernelGGL((nl_partial_kernel<T, CPLX>), dim3(L.nchunks, nct), dim3(256), 0, s,
                     L.chunk_atom, L.chunk_begin, L.atom_ptr, L.atom_node, L.atom_val,
                     static_cast<const T*>(L.X), L.ldx, L.ncols, static_cast<T*>(L.partial), L.ldhp);
  const int nreal = CPLX ? 2 * L.ncols : L.ncols;
  hipLaunchKernelGGL((nl_reduce_kernel<T>), dim3(L.natoms * 4, (L.ldhp + 255) / 256), dim3(256), 0, s,
                     L.atom_chunk_ptr, L.hcoef, static_cast<const T*>(L.partial), static_cast<T*>(L.hP),
                     L.ldhp, nreal);
  return hipGetLastError();
}

// ---- elementwise helpers ----------------------------------------------------
template <typename T>
__global__ void fill_kernel(T* dst, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t total = rows * cols;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = i / cols, c = i % cols;
    dst[r * ld + c] = T(0);
  }
}

// dst[r][c] = src[r][c] for a rows x cols block.  Blocks of at most 256
// columns: each workgroup step covers 256 / cols whole rows (thread = row in
// the step, column), so no thread divides a 64-bit index; wider blocks: one
// row per step, columns strided by 256.
template <typename TD, typename TS>
__global__ void __launch_bounds__(256) convert_kernel(TD* dst, int64_t ldd, const TS* src, int64_t lds,
                                                      int64_t rows, int ncol) {
  if (ncol <= 256) {
    const int rpb = 256 / ncol;
    const int tr = threadIdx.x / ncol, c = threadIdx.x % ncol;
    if (tr >= rpb) return;
    const int64_t step = static_cast<int64_t>(gridDim.x) * rpb;
#pragma unroll 4
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * rpb + tr; r < rows; r += step)
      dst[r * ldd + c] = static_cast<TD>(src[r * lds + c]);
  } else {
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
      for (int c = threadIdx.x; c < ncol; c += 256) dst[r * ldd + c] = static_cast<TD>(src[r * lds + c]);
  }
}

inline bool is_double(int prec) { return prec == CHFSI_F64 || prec == CHFSI_C128; }

unsigned grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return static_cast<unsigned>(g);
}

}  // namespace

hipError_t launch_nl_project(const NlLaunch& L, int prec, hipStream_t s) {
  switch (prec) {
    case CHFSI_F64: return nl_launch<double, false>(L, s);
    case CHFSI_F32:
    case CHFSI_BF16: return nl_launch<float, false>(L, s);
    case CHFSI_C128: return nl_launch<double, true>(L, s);
    case CHFSI_C64: return nl_launch<float, true>(L, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_nl_project_batched(const NlBatch& b, int prec, hipStream_t s) {
  if (b.nprob <= 0 || b.total_chunks <= 0) return hipSuccess;
  const dim3 gp(static_cast<unsigned>(b.total_chunks), static_cast<unsigned>(b.max_col_tiles));
  const dim3 gr(static_cast<unsigned>(b.total_rows), static_cast<unsigned>(b.max_row_blocks));
  const NlLaunch* d = static_cast<const NlLaunch*>(b.descs);
  switch (prec) {
    case CHFSI_F64:
      hipLaunchKernelGGL((nl_partial_batched_kernel<double, false>), gp, dim3(256), 0, s, d, b.chunk_off, b.nprob);
      hipLaunchKernelGGL((nl_reduce_batched_kernel<double, false>), gr, dim3(256), 0, s, d, b.row_off, b.nprob);
      break;
    case CHFSI_F32:
      hipLaunchKernelGGL((nl_partial_batched_kernel<float, false>), gp, dim3(256), 0, s, d, b.chunk_off, b.nprob);
      hipLaunchKernelGGL((nl_reduce_batched_kernel<float, false>), gr, dim3(256), 0, s, d, b.row_off, b.nprob);
      break;
    case CHFSI_C128:
      hipLaunchKernelGGL((nl_partial_batched_kernel<double, true>), gp, dim3(256), 0, s, d, b.chunk_off, b.nprob);
      hipLaunchKernelGGL((nl_reduce_batched_kernel<double, true>), gr, dim3(256), 0, s, d, b.row_off, b.nprob);
      break;
    case CHFSI_C64:
      hipLaunchKernelGGL((nl_partial_batched_kernel<float, true>), gp, dim3(256), 0, s, d, b.chunk_off, b.nprob);
      hipLaunchKernelGGL((nl_reduce_batched_kernel<float, true>), gr, dim3(256), 0, s, d, b.row_off, b.nprob);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill(void* dst, int64_t rows, int64_t cols, int64_t ld, int prec, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const unsigned g = grid_for(rows * cols);
  if (is_double(prec))
    hipLaunchKernelGGL(fill_kernel<double>, dim3(g), dim3(256), 0, s, static_cast<double*>(dst), rows, cols, ld);
  else
    hipLaunchKernelGGL(fill_kernel<float>, dim3(g), dim3(256), 0, s, static_cast<float*>(dst), rows, cols, ld);
  return hipGetLastError();
}

hipError_t launch_convert(void* dst, int64_t ldd, int dprec, const void* src, int64_t lds, int sprec,
                          int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (cols > 0x7fffffff) return hipErrorInvalidValue;
  const unsigned g = grid_for(rows * cols);
  const bool dd = is_double(dprec), sd = is_double(sprec);
  const int ncol = static_cast<int>(cols);
  if (dd && sd)
    hipLaunchKernelGGL((convert_kernel<double, double>), dim3(g), dim3(256), 0, s, static_cast<double*>(dst), ldd,
                       static_cast<const double*>(src), lds, rows, ncol);
  else if (dd && !sd)
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(g), dim3(256), 0, s, static_cast<double*>(dst), ldd,
                       static_cast<const float*>(src), lds, rows, ncol);
  else if (!dd && sd)
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(g), dim3(256), 0, s, static_cast<float*>(dst), ldd,
                       static_cast<const double*>(src), lds, rows, ncol);
  else
    hipLaunchKernelGGL((convert_kernel<float, float>), dim3(g), dim3(256), 0, s, static_cast<float*>(dst), ldd,
                       static_cast<const float*>(src), lds, rows, ncol);
  return hipGetLastError();
}

// ---- fixed scratch for the allocation-free H~.X ------------------------------
// The projector partials and coefficients of chfsi_apply_noalloc() live in
// this file-scope device array instead of context workspace.  Each device the
// library runs on holds its own copy (kScratchBytes) until the process ends.
// Host code must never pass the array's name to a kernel: in host code it is
// a host-side stand-in, not a device address.  scratch_address() resolves the
// address for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** out) {
  *out = nullptr;
  return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

}  // namespace chfsi
