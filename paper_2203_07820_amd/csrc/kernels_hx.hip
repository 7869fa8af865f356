// Cell-wise H~.X on gfx950 (DFT-FE 1.0, Section 4.3, Eq. celldgemm and
// Algorithm 4), fused with one step of the scaled Chebyshev recurrence
// (Section 3.1).
//
// One workgroup owns one hexahedral cell and a 64-wide tile of columns.  It
//   1. reads the cell's nodal rows X^c (node-major, 64 contiguous values per
//      node) straight into MFMA B-operand registers;
//   2. multiplies the shared reference cell matrix A (mcell x mcell, streamed
//      from L2 in MFMA operand order) by X^c with 16x16x4 MFMA (f64 or f32;
//      16x16x32 bf16 with f32 accumulation for the bf16 variant),
//      accumulating in registers; for complex operators A_r X + A_i X' where
//      X' is X with (re, im) -> (-im, re);
//   3. adds the nonlocal term C^{c,a} (h P_a) for every atom a whose
//      projectors touch the cell, as extra 4-wide k steps (Algorithm 4 steps
//      5-6, with P_a from the node-level contraction of kernels_nl.hip);
//   4. scatters alpha * Y^c into the target with atomic adds (ASEMB_FEM;
//      plain stores for nodes interior to the cell, which have no other
//      contributor).  The owner cell of each node (local indices all < p) adds
//      alpha (V_j - c) X_k[j] - beta X_{k-1}[j], so the target ends up holding
//      X_{k+1} = alpha (H~ X_k - c X_k) - beta X_{k-1} without a separate pass;
//      the owner then zeroes X_{k-1}[j], which becomes the target two steps on
//      (nodes interior to the cell excepted: their value is stored, not added).
//
// Node numbering: n = ncell * p nodes per direction, node (ix, iy, iz) has id
// ix + n (iy + n iz); cell (cx, cy, cz) local node (a, b, c) is global node
// ((cx p + a) mod n, ...).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "device_util.h"
#include "internal.h"

namespace chfsi {
namespace {

constexpr int kNT = 64;     // columns per workgroup tile

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <typename T> struct Mma;
// Operand layouts (both types): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Accumulator register i of lane l holds D[row][l % 16]
// with row = 4 i + l / 16 for f64 and row = 4 (l / 16) + i for f32.
template <> struct Mma<double> {
  typedef d4 acc_t;
  __device__ __forceinline__ static acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int i) { return 4 * i + lane / 16; }
};
template <> struct Mma<float> {
  typedef f4 acc_t;
  __device__ __forceinline__ static acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int i) { return 4 * (lane / 16) + i; }
};
// bf16 16x16x32 with f32 accumulation: lane l supplies A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16], j = 0..7; the accumulator layout is that of
// the f32 16x16x4 MFMA, so both kinds can accumulate into the same tile.
__device__ __forceinline__ f4 mma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}


// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD works on a contiguous range of cells (neighbouring cells share nodes,
// which then hit the same L2).
__device__ __forceinline__ int xcd_remap(int pid, int nblk) {
  const int q = nblk / 8, r = nblk % 8;
  const int xcd = pid % 8, slot = pid / 8;
  return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

template <typename T>
struct HxArgs {
  const T* A;       // cell matrix, 16x16x4 A-operand order [row tile][k step][lane]
  const T* Ai;      // imaginary part (complex operators)
  const bf8* Ab;    // bf16 copy, 16x16x32 A-operand order [row tile][k step][lane]
  const double* vdiag;
  const T* Xk;
  const T* Xp;
  T* Tg;
  int64_t ldx, ldp, ldt;
  int ncols, nc;
  int zero_prev;
  T alpha, c, beta;
  const int32_t* pair_ptr;
  const int32_t* pair_atom;
  const T* pair_re;
  const T* pair_im;
  const T* hP;
  int64_t ldhp;
  int64_t astride;  // elements between the real cell matrices of consecutive cells (0: one shared)
  // deterministic assembly: this launch covers only the cells cells[0..ncell)
  // (one colour class, no two of which share a node); null: every cell
  const int32_t* cells;
  int ncell;
};

// Work item bid of a single-problem launch: its cell and first column.  With
// a colour class, work item bid takes the class's cell bid % ncell.
template <int NT, typename T>
__device__ __forceinline__ void item_of(const HxArgs<T>& a, const int bid, int& cell, int& col0) {
  const int E = a.nc * a.nc * a.nc;
  const int ne = a.cells ? a.ncell : E;
  const int i = bid % ne;
  cell = a.cells ? to_global(a.cells)[i] : i;
  col0 = (bid / ne) * NT;
}

// Buffer resource over `bytes` bytes at p (raw buffer, 32-bit words).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <> __device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ bf8 buf_load<bf8>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(bf8, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// Per-cell row tables in LDS, written once per work item: xoff[l] = element
// offset of cell row l in X (node id * ldx; row 0's for padding rows) and
// gid[l] = node id | owner << 30 | interior << 29 (-1 for padding rows).  The
// owner of a node is the cell in which its local indices are all < p; an
// interior node (all local indices in [1, p-1]) belongs to this cell only.
template <int MP, typename T> struct RowTables {
  int64_t xoff[MP];
  int32_t gid[MP];
  T wv[MP];     // alpha (V_j - c) for owned rows, 0 otherwise
};

// Fills the per-cell row tables of `cell` (threads tid, tid + nthr, ...).
template <int P, typename T>
__device__ __forceinline__ void row_tables(const HxArgs<T>& a, const int cell, const int tid, const int nthr,
                                           RowTables<(((P + 1) * (P + 1) * (P + 1) + 15) / 16 * 16), T>& tab) {
  constexpr int Q = P + 1;
  constexpr int MC = Q * Q * Q;
  constexpr int MP = (MC + 15) / 16 * 16;
  const int nc = a.nc, n = nc * P;
  const int cx = cell % nc, cy = (cell / nc) % nc, cz = cell / (nc * nc);
  for (int l = tid; l < MP; l += nthr) {
    int32_t g = -1;
    int64_t off = 0;
    T w = T(0);
    if (l < MC) {
      const int la = l % Q, lb = (l / Q) % Q, lc = l / (Q * Q);
      int gx = cx * P + la; if (gx >= n) gx -= n;
      int gy = cy * P + lb; if (gy >= n) gy -= n;
      int gz = cz * P + lc; if (gz >= n) gz -= n;
      const int32_t node = gx + n * (gy + n * gz);
      off = static_cast<int64_t>(node) * a.ldx;
      const bool inner = la > 0 && la < P && lb > 0 && lb < P && lc > 0 && lc < P;
      const bool owner = la < P && lb < P && lc < P;
      g = node | (owner ? (1 << 30) : 0) | (inner ? (1 << 29) : 0);
      if (owner) w = a.alpha * (static_cast<T>(to_global(a.vdiag)[node]) - a.c);
    }
    tab.xoff[l] = off;
    tab.gid[l] = g;
    tab.wv[l] = w;
  }
}

// The part of a work item after the cell products, shared by the cell
// kernels: the nonlocal term C^{c,a} (h P_a) of every (cell, atom) pair as
// extra 4-wide k steps into the accumulators, then the epilogue (scaling, the
// owner's diagonal and recurrence terms, assembly).  The wave owns row tiles
// rt0 .. rt0 + RPW - 1 and column tiles ct0 .. ct0 + CPW - 1 (16 x 16 each)
// of the item's columns [col0, col0 + 64); acc holds its accumulators in the
// 16x16x4 layout.
// nonlocal: Y^c += C^{c,a} (h P_a) for the atoms touching this cell, one
// 4-wide k step per (cell, atom) pair
template <int MP, typename T, bool CPLX, int RPW, int CPW>
__device__ __forceinline__ void cell_nonlocal(const HxArgs<T>& a, typename Mma<T>::acc_t (&acc)[RPW][CPW],
                                              const int cell, const int col0, const int rt0, const int ct0,
                                              const int lane) {
  constexpr int RT = MP / 16;
  if (a.pair_ptr != nullptr) {
    const gptr<const int32_t> pp = to_global(a.pair_ptr);
    const int p0 = pp[cell], p1 = pp[cell + 1];
    for (int pr = p0; pr < p1; ++pr) {
      const int at = to_global(a.pair_atom)[pr];
      const gptr<const T> hrow = to_global(a.hP) + (static_cast<int64_t>(at) * 4 + lane / 16) * a.ldhp + col0;
      T b[CPW], bs[CPW], cv[RPW], ci[CPLX ? RPW : 1];
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int cc = (ct0 + c) * 16 + lane % 16;
        b[c] = hrow[cc];
        if constexpr (CPLX) {
          const T o = hrow[cc ^ 1];
          bs[c] = (cc & 1) ? o : -o;
        }
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        cv[r] = to_global(a.pair_re)[(static_cast<int64_t>(pr) * RT + rt0 + r) * 64 + lane];
        if constexpr (CPLX) ci[r] = to_global(a.pair_im)[(static_cast<int64_t>(pr) * RT + rt0 + r) * 64 + lane];
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          acc[r][c] = Mma<T>::run(cv[r], b[c], acc[r][c]);
          if constexpr (CPLX) acc[r][c] = Mma<T>::run(ci[r], bs[c], acc[r][c]);
        }
    }
  }
}

// The nonlocal term for real operators with the operands of the next pair in
// flight while the current pair multiplies (loop unrolled by 2 so that each
// operand buffer keeps a fixed role).  `first` holds the first pair's
// operands, loaded by the caller (before its k loop) with nl_load.
template <typename T, int RPW, int CPW> struct NlOps { T b[CPW], cv[RPW]; };
template <int MP, typename T, int RPW, int CPW>
__device__ __forceinline__ void nl_load(const HxArgs<T>& a, const int pr, const int col0, const int rt0,
                                        const int ct0, const int lane, NlOps<T, RPW, CPW>& o) {
  constexpr int RT = MP / 16;
  const int at = to_global(a.pair_atom)[pr];
  const gptr<const T> hrow = to_global(a.hP) + (static_cast<int64_t>(at) * 4 + lane / 16) * a.ldhp + col0;
#pragma unroll
  for (int c = 0; c < CPW; ++c) o.b[c] = hrow[(ct0 + c) * 16 + lane % 16];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
    o.cv[r] = to_global(a.pair_re)[(static_cast<int64_t>(pr) * RT + rt0 + r) * 64 + lane];
}
template <int MP, typename T, int RPW, int CPW>
__device__ __forceinline__ void cell_nonlocal_pf(const HxArgs<T>& a, typename Mma<T>::acc_t (&acc)[RPW][CPW],
                                                 const int p0, const int p1, const int col0, const int rt0,
                                                 const int ct0, const int lane, NlOps<T, RPW, CPW>& first) {
  auto mma = [&](const NlOps<T, RPW, CPW>& o) {
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc[r][c] = Mma<T>::run(o.cv[r], o.b[c], acc[r][c]);
  };
  NlOps<T, RPW, CPW> second;
  for (int pr = p0; pr < p1; pr += 2) {
    if (pr + 1 < p1) nl_load<MP, T, RPW, CPW>(a, pr + 1, col0, rt0, ct0, lane, second);
    mma(first);
    if (pr + 1 < p1) {
      if (pr + 2 < p1) nl_load<MP, T, RPW, CPW>(a, pr + 2, col0, rt0, ct0, lane, first);
      mma(second);
    }
  }
}

template <int MP, typename T, bool CPLX, int RPW, int CPW, int ED, int SR = (sizeof(T) == 8 ? 2 : 4)>
__device__ __forceinline__ void cell_tail(const HxArgs<T>& a, typename Mma<T>::acc_t (&acc)[RPW][CPW], const int cell,
                                          const int col0, const int rt0, const int ct0, const int lane,
                                          RowTables<MP, T>& tab) {
  cell_nonlocal<MP, T, CPLX, RPW, CPW>(a, acc, cell, col0, rt0, ct0, lane);

  // epilogue: scale, owner terms, atomic assembly.  Per row tile, every
  // lane loads its owner operands (X_k, X_{k-1}) without branches, at
  // addresses that are valid for every lane: rows this cell does not own (and
  // padding rows) read node 0's row, which stays in cache, columns beyond
  // ncols read column ncols - 1.  The loads of tile r + 1 are issued before
  // the stores and atomics of tile r, so that their latency overlaps; the
  // selects discard what non-owners read, and only stores and atomics are
  // masked.  alpha (V - c) of owned rows comes from the LDS table.
  const gptr<const T> __restrict__ Xk = to_global(a.Xk);
  const gptr<T> __restrict__ Xp = to_global(const_cast<T*>(a.Xp));
  const gptr<T> __restrict__ Tg = to_global(a.Tg);
  const bool has_prev = a.Xp != nullptr;
  int colc[CPW];
  bool colok[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int col = col0 + (ct0 + c) * 16 + lane % 16;
    colok[c] = col < a.ncols;
    colc[c] = colok[c] ? col : a.ncols - 1;
  }
  // stages of SR of the 4 accumulator rows of each lane: by default half a
  // row tile for 8-byte values (whole tiles would not fit next to the FP64
  // accumulators), a whole tile for 4-byte values
  static_assert(SR == 2 || SR == 4, "epilogue stage rows");
  struct Ops {
    int32_t g[SR];
    T xk[SR][CPW], xp[SR][CPW];
  };
  auto fetch = [&](int h, Ops& o) {
    const int r = h / (4 / SR);
#pragma unroll
    for (int k = 0; k < SR; ++k) {
      const int i = (h % (4 / SR)) * SR + k;
      o.g[k] = tab.gid[(rt0 + r) * 16 + Mma<T>::row(lane, i)];
      const int64_t go = (o.g[k] >= 0 && (o.g[k] & (1 << 30))) ? (o.g[k] & ((1 << 29) - 1)) : 0;
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        o.xk[k][c] = Xk[go * a.ldx + colc[c]];
        o.xp[k][c] = has_prev ? Xp[go * a.ldp + colc[c]] : T(0);
      }
    }
  };
  auto finish = [&](int h, const Ops& o) {
    const int r = h / (4 / SR);
#pragma unroll
    for (int k = 0; k < SR; ++k) {
      const int i = (h % (4 / SR)) * SR + k;
      const int32_t g = o.g[k];
      const bool valid = g >= 0;
      const bool own = valid && (g & (1 << 30));
      const bool inner = valid && (g & (1 << 29));
      const int64_t gn = valid ? (g & ((1 << 29) - 1)) : 0;
      const T vc = tab.wv[(rt0 + r) * 16 + Mma<T>::row(lane, i)];
      const T bp = own ? a.beta : T(0);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const T v = a.alpha * acc[r][c][i] + vc * o.xk[k][c] - bp * o.xp[k][c];
        // the owner clears X_{k-1}[j] for the step that targets this buffer
        // two steps on; an interior node needs no clearing, since its single
        // contributor will store (not add) its value there
        if (own && !inner && has_prev && a.zero_prev && colok[c]) Xp[gn * a.ldp + colc[c]] = T(0);
        // the target starts at zero and an interior node has no other
        // contributor: a plain store is the sum
        if (inner && colok[c]) Tg[gn * a.ldt + colc[c]] = v;
        else if (valid && colok[c]) atomic_add(Tg + gn * a.ldt + colc[c], v);
      }
    }
  };
  // the operands of stage h + ED - 1 are in flight while stage h is
  // finished (ED = 3 fits for 8-byte values, whose main-loop operand
  // registers are free by now, except in the item loop of the chunked
  // batched kernel)
  static_assert(ED == 2 || ED == 3, "epilogue depth");
  constexpr int NH = (4 / SR) * RPW;   // stages (odd when SR = 4 and RPW is odd)
  Ops o[ED];
#pragma unroll
  for (int h = 0; h < ED - 1 && h < NH; ++h) fetch(h, o[h]);
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    if (h + ED - 1 < NH) fetch(h + ED - 1, o[(h + ED - 1) % ED]);
    finish(h, o[h % ED]);
  }
}

// One work item: cell `cell`, columns [col0, col0 + NT) (NT = 64 or 32).
//
// Work split inside a workgroup: WAVES/CG row groups x CG column groups.  The
// number of 16-row tiles is even for every order p in [2, 7], so each wave
// owns RT / (WAVES/CG) row tiles and NT/16/CG column tiles, with no guards.
// The 64-column tile takes CG = 2 by default; CG = 1 (each wave all 64
// columns, so each A fragment serves four column tiles) where the
// accumulators fit beside the pipeline (real FP32, p <= 6): the 32-cycle FP32
// MFMA leaves half the time of the FP64 one to hide the same operand loads.
// The 32-column tile (CG = 1, two column tiles per wave, half the waves per
// workgroup) halves the padding of blocks of at most 32 columns and doubles
// the number of work items.
// B fragments are read straight from global memory into registers (no LDS
// staging of X, no barriers in the loop): in a 4-wide k step, lanes
// 16 q .. 16 q + 15 read 16 consecutive columns of cell row 4 kg + q, one
// cache line per 16 lanes, at the row offset kept in the LDS table.  A
// fragments come through buffer loads whose per-row-tile offsets live in
// scalar registers; they are loaded one k step ahead and B fragments two
// (HBM latency), the A load of the next step issued before the B load two
// steps ahead, so that the in-order vector-memory counter never makes an MFMA
// wait on HBM.  Column lanes beyond ncols read a valid column and are never
// stored; padding rows (l >= mcell) are zeroed.
template <int P, typename T, bool CPLX, int WAVES, int ED, int CG = 2, int NT = kNT>
__device__ __forceinline__ void cell_item(const HxArgs<T>& a, const int cell, const int col0,
                                          RowTables<(((P + 1) * (P + 1) * (P + 1) + 15) / 16 * 16), T>& tab) {
  constexpr int Q = P + 1;
  constexpr int MC = Q * Q * Q;
  constexpr int MP = (MC + 15) / 16 * 16;
  constexpr int RT = MP / 16;           // row tiles
  constexpr int KS = MP / 4;            // 4-wide k steps
  constexpr int RG = WAVES / CG;        // row groups
  constexpr int RPW = RT / RG;          // row tiles per wave
  constexpr int CPW = NT / 16 / CG;     // column tiles per wave
  static_assert(RT % RG == 0 && KS % 2 == 0 && WAVES % CG == 0, "tiling");
  using acc_t = typename Mma<T>::acc_t;

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int lane = tid % 64;
  const int rt0 = (wave / CG) * RPW, ct0 = (wave % CG) * CPW;

  // row tables (the barrier in front protects the previous item's readers)
  __syncthreads();
  row_tables<P, T>(a, cell, tid, 64 * WAVES, tab);
  __syncthreads();

  acc_t acc[RPW][CPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int c = 0; c < CPW; ++c) acc[r][c] = acc_t{0, 0, 0, 0};

  // per-lane column pointers, clamped to a valid column; complex blocks keep
  // the lane's parity (re/im) so that the partner column cc ^ 1 stays valid
  // (their ncols, counted in reals, is even)
  gptr<const T> xcol[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    int cc = col0 + (ct0 + c) * 16 + lane % 16;
    if (cc >= a.ncols) cc = CPLX ? a.ncols - 2 + (lane & 1) : a.ncols - 1;
    xcol[c] = to_global(a.Xk) + cc;
  }

  // A fragments of this wave: tile (rt0 + r, k step kg) at element
  // ((rt0 + r) KS + kg) 64 + lane
  constexpr int RI = CPLX ? RPW : 1;
  constexpr int CI = CPLX ? CPW : 1;
  const uint32_t abytes = static_cast<uint32_t>(RT) * KS * 64 * sizeof(T);
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(a.A + static_cast<int64_t>(cell) * a.astride, abytes);
  const __amdgpu_buffer_rsrc_t rai = make_rsrc(CPLX ? a.Ai : a.A, abytes);
  int soff[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) soff[r] = __builtin_amdgcn_readfirstlane((rt0 + r) * KS * 64 * static_cast<int>(sizeof(T)));
  // both loaders clamp the k step to the last one, so that the pipeline's
  // loads past the end (never used) read valid memory without a branch
  auto load_a = [&](T (&av)[RPW], T (&avi)[RI], int kg) {
    const int vo = ((kg < KS ? kg : KS - 1) * 64 + lane) * static_cast<int>(sizeof(T));
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      av[r] = buf_load<T>(ra, vo, soff[r]);
      if constexpr (CPLX) avi[r] = buf_load<T>(rai, vo, soff[r]);
    }
  };
  auto load_b = [&](T (&bv)[CPW], T (&bo)[CI], int kg) {
    const int l = (kg < KS ? kg : KS - 1) * 4 + lane / 16;
    const int64_t off = tab.xoff[l];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      bv[c] = xcol[c][off];
      // the partner (re <-> im) of column cc is cc ^ 1, one element away
      if constexpr (CPLX) bo[c] = xcol[c][off + ((lane & 1) ? -1 : 1)];
    }
  };
  // padding rows (>= mcell) of step kg are zeroed here, at use, so that no
  // wait is forced at the load
  auto compute = [&](const T (&av)[RPW], const T (&avi)[RI], const T (&bin)[CPW], const T (&boin)[CI], int kg) {
    T bv[CPW], bo[CI], bs[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      bv[c] = bin[c];
      if constexpr (CPLX) bo[c] = boin[c];
    }
    if ((kg + 1) * 4 > MC) {
      const bool ok = kg * 4 + lane / 16 < MC;
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        bv[c] = ok ? bv[c] : T(0);
        if constexpr (CPLX) bo[c] = ok ? bo[c] : T(0);
      }
    }
    if constexpr (CPLX) {
#pragma unroll
      for (int c = 0; c < CPW; ++c) bs[c] = (lane & 1) ? bo[c] : -bo[c];
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        acc[r][c] = Mma<T>::run(av[r], bv[c], acc[r][c]);
        if constexpr (CPLX) acc[r][c] = Mma<T>::run(avi[r], bs[c], acc[r][c]);
      }
  };
  // Pipeline: the A fragments of step s + 1 and the B rows of step s + 2
  // are in flight while step s multiplies.  The loop is unrolled by 4 so
  // that every buffer keeps a fixed role (A period 2, B period 4): a copy
  // between buffers would make the compiler wait for the loads in flight
  // into the source buffer, draining the pipeline every iteration.
  static_assert(KS % 4 == 0, "k steps come in groups of 4");
  T aq[2][RPW], aiq[2][RI];
  T bq[4][CPW], oq[4][CI];
  load_b(bq[0], oq[0], 0);
  load_a(aq[0], aiq[0], 0);
  load_b(bq[1], oq[1], 1);
  for (int kg = 0; kg < KS; kg += 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = kg + j;
      load_a(aq[(j + 1) % 2], aiq[(j + 1) % 2], s + 1);
      load_b(bq[(j + 2) % 4], oq[(j + 2) % 4], s + 2);
      compute(aq[j % 2], aiq[j % 2], bq[j], oq[j], s);
      // keep each step's loads behind the previous step's MFMAs: hoisted
      // further, they would hold a third A buffer and spill at FP64
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // 4-byte values with four column tiles per wave: epilogue stages of half a
  // row tile, so that the stages fit beside the accumulators
  constexpr int SR = (sizeof(T) == 8 || CPW > 2) ? 2 : 4;
  cell_tail<MP, T, CPLX, RPW, CPW, ED, SR>(a, acc, cell, col0, rt0, ct0, lane, tab);
}

// Column groups per workgroup of the 64-column tile (see cell_item).
template <int P, typename T, bool CPLX> constexpr int col_groups() {
  return (!CPLX && sizeof(T) == 4 && P <= 6) ? 1 : 2;
}
template <int P> constexpr int rows_padded() { return ((P + 1) * (P + 1) * (P + 1) + 15) / 16 * 16; }
// epilogue stages in flight + 1
template <typename T> constexpr int epilogue_depth() { return sizeof(T) == 8 ? 3 : 2; }

// Single problem: one workgroup per (cell, column tile), cells fastest.
template <int P, typename T, bool CPLX, int WAVES, int OCC, int CG, int NT>
__global__ void __attribute__((amdgpu_flat_work_group_size(64 * WAVES, 64 * WAVES), amdgpu_waves_per_eu(OCC, OCC)))
cell_hx_kernel(const HxArgs<T> a) {
  __shared__ RowTables<rows_padded<P>(), T> tab;
  int cell, col0;
  item_of<NT>(a, xcd_remap(blockIdx.x, gridDim.x), cell, col0);
  cell_item<P, T, CPLX, WAVES, epilogue_depth<T>(), CG, NT>(a, cell, col0, tab);
}

// bf16 cell products with FP32 iterates (the BF16 filter precision).  The
// FP64/FP32 item above streams its B fragments from memory, each wave reading
// its own; at 16 cycles per bf16 MFMA that leaves the main loop waiting on
// memory and each A fragment (read from L2) serving only 2 column tiles.
// Here a workgroup of MP / 32 waves owns one (cell, 64-column) item:
//   1. the cell block X^c is staged once into LDS, rounded to bf16 (nearest
//      even) and stored column-major (bt[col * CS + row], CS = MP + 8, so
//      that the 16 lanes of a 16-byte LDS read hit 16 distinct 4-bank
//      groups), with every wave's row loads in flight together (lane =
//      column, 16 row pairs per wave); an FP32 copy (xs, p <= 6) keeps X_k
//      for the owner's diagonal term;
//   2. X_{k-1} at the owned rows of each wave's accumulators and the first
//      (cell, atom) pair's operands are loaded before the k loop, so that
//      the nonlocal term and the epilogue wait on nothing but their own
//      later pairs;
//   3. each wave multiplies 2 row tiles (32 rows) of A by all 4 column tiles,
//      A fragments from L2 two k steps ahead (each used 4 times), B
//      fragments from LDS with one 16-byte read per column tile;
//   4. nonlocal term, then the epilogue (scaling, owner terms, assembly) with
//      2 row tiles x 4 column tiles per wave.
// Measured on the c1 operator (128-column filter step): 2.07 ms against
// 2.94 ms for the bf16 variant of the FP32 item.  Rejected: a persistent
// form with a loader wave streaming the next item into LDS (2.6-3.2 ms: on
// gfx9 stores count in the same in-order counter as loads, so the compute
// waves' first load of an item waited for the previous item's stores);
// an FP32 output tile in LDS so that every store covers a whole row
// (2.18 ms); dropping the LDS copy for two workgroups per CU (2.30 ms).
template <int P> constexpr int bf16_waves() { return rows_padded<P>() / 32; }

template <int P>
__global__ void __attribute__((amdgpu_flat_work_group_size(64 * bf16_waves<P>(), 64 * bf16_waves<P>())))
cell_hx_bf16_kernel(const HxArgs<float> a) {
  constexpr int Q = P + 1;
  constexpr int MC = Q * Q * Q;
  constexpr int MP = rows_padded<P>();
  constexpr int RT = MP / 16;           // row tiles
  constexpr int KB = MP / 32;           // 32-wide k steps
  constexpr int NW = bf16_waves<P>();   // waves: 2 row tiles each
  constexpr int RPW = 2, CPW = kNT / 16;
  constexpr int CS = MP + 8;            // LDS column stride of the bf16 block (elements)
  constexpr int SB = 8;                 // row pairs per batch of staging loads
  constexpr int AD = 3;                 // A fragments in flight (k steps ahead + 1)
  static_assert(MP % 32 == 0 && RT == NW * RPW, "bf16 tiling");
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  // FP32 copy of X^c, row-major with a row stride of 68 floats (the 4 rows of
  // one accumulator access fall in distinct banks), while it fits (p <= 6)
  constexpr int XS = kNT + 4;
  constexpr bool XS_LDS = (MP * XS * 4 + kNT * CS * 2 + MP * 16) <= 160 * 1024;
  __shared__ RowTables<MP, float> tab;
  __shared__ __attribute__((aligned(16))) __bf16 bt[kNT * CS];
  __shared__ float xs[XS_LDS ? MP * XS : 1];

  int cell, col0;
  item_of<kNT>(a, xcd_remap(blockIdx.x, gridDim.x), cell, col0);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int lane = tid % 64;
  row_tables<P, float>(a, cell, tid, 64 * NW, tab);
  __syncthreads();

  // 1. stage X^c (column col0 + lane, clamped to a valid column); rows >= MC
  //    read node 0 and are replaced by zeros in bt
  {
    int cc = col0 + lane;
    if (cc >= a.ncols) cc = a.ncols - 1;
    const float* __restrict__ xcol = a.Xk + cc;
#pragma unroll
    for (int h = 0; h < 16; h += SB) {
      float v[2 * SB];
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        const int l0 = 2 * (wave + NW * (h + i));
        v[2 * i] = xcol[tab.xoff[l0]];
        v[2 * i + 1] = xcol[tab.xoff[l0 + 1]];
      }
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        const int l0 = 2 * (wave + NW * (h + i));
        bf2 pr;
        pr[0] = static_cast<__bf16>(l0 < MC ? v[2 * i] : 0.f);
        pr[1] = static_cast<__bf16>(l0 + 1 < MC ? v[2 * i + 1] : 0.f);
        *reinterpret_cast<bf2*>(&bt[lane * CS + l0]) = pr;
        if constexpr (XS_LDS) {
          xs[l0 * XS + lane] = v[2 * i];
          xs[(l0 + 1) * XS + lane] = v[2 * i + 1];
        }
      }
    }
  }
  __syncthreads();

  // 2. X_{k-1} at the owned rows of this wave's accumulators (16x16x4 layout:
  //    row 16 (rt0 + r) + 4 (lane / 16) + i, column 16 c + lane % 16); rows
  //    this cell does not own read node 0's row and are discarded
  const int rt0 = wave * RPW;
  int colc[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int col = col0 + c * 16 + lane % 16;
    colc[c] = col < a.ncols ? col : a.ncols - 1;
  }
  const bool has_prev = a.Xp != nullptr;
  float xp[RPW][4][CPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int32_t g = tab.gid[(rt0 + r) * 16 + 4 * (lane / 16) + i];
      const int64_t go = (has_prev && g >= 0 && (g & (1 << 30))) ? (g & ((1 << 29) - 1)) : 0;
#pragma unroll
      for (int c = 0; c < CPW; ++c) xp[r][i][c] = has_prev ? a.Xp[go * a.ldp + colc[c]] : 0.f;
    }
  const int p0 = a.pair_ptr != nullptr ? a.pair_ptr[cell] : 0;
  const int p1 = a.pair_ptr != nullptr ? a.pair_ptr[cell + 1] : 0;
  NlOps<float, RPW, CPW> nl0;
  if (p0 < p1) nl_load<MP, float, RPW, CPW>(a, p0, col0, rt0, 0, lane, nl0);

  // 3. cell products: rows 32 wave .. 32 wave + 31, all 64 columns
  f4 acc[RPW][CPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int c = 0; c < CPW; ++c) acc[r][c] = f4{0, 0, 0, 0};
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(a.Ab, static_cast<uint32_t>(RT) * KB * 64 * 16);
  int soff[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) soff[r] = __builtin_amdgcn_readfirstlane((rt0 + r) * KB * 64 * 16);
  auto load_a = [&](bf8 (&av)[RPW], int kg) {
    const int vo = (kg * 64 + lane) * 16;
#pragma unroll
    for (int r = 0; r < RPW; ++r) av[r] = buf_load<bf8>(ra, vo, soff[r]);
  };
  const __bf16* bcol = bt + (lane % 16) * CS + 8 * (lane / 16);
  bf8 aq[AD][RPW];
#pragma unroll
  for (int k = 0; k < AD - 1 && k < KB; ++k) load_a(aq[k], k);
#pragma unroll
  for (int kg = 0; kg < KB; ++kg) {
    if (kg + AD - 1 < KB) load_a(aq[(kg + AD - 1) % AD], kg + AD - 1);
    bf8 bq[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) bq[c] = *reinterpret_cast<const bf8*>(bcol + c * 16 * CS + kg * 32);
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc[r][c] = mma_bf16(aq[kg % AD][r], bq[c], acc[r][c]);
  }

  // 4. nonlocal term, then the epilogue: X_k from the LDS copy (memory for
  //    p = 7), X_{k-1} from the registers loaded above
  cell_nonlocal_pf<MP, float, RPW, CPW>(a, acc, p0, p1, col0, rt0, 0, lane, nl0);
  const gptr<float> __restrict__ Xp = to_global(const_cast<float*>(a.Xp));
  const gptr<float> __restrict__ Tg = to_global(a.Tg);
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = (rt0 + r) * 16 + 4 * (lane / 16) + i;
      const int32_t g = tab.gid[row];
      const bool valid = g >= 0;
      const bool own = valid && (g & (1 << 30));
      const bool inner = valid && (g & (1 << 29));
      const int64_t gn = valid ? (g & ((1 << 29) - 1)) : 0;
      const float vc = tab.wv[row];
      const float bp = own ? a.beta : 0.f;
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const bool ok = col0 + c * 16 + lane % 16 < a.ncols;
        float xk;
        if constexpr (XS_LDS) xk = xs[row * XS + c * 16 + lane % 16];
        else xk = a.Xk[(own ? gn : 0) * a.ldx + colc[c]];
        const float v = a.alpha * acc[r][c][i] + vc * xk - bp * xp[r][i][c];
        // as in cell_tail: clear X_{k-1} for reuse as a target (interior
        // nodes excepted), store interior nodes, add the others
        if (own && !inner && has_prev && a.zero_prev && ok) Xp[gn * a.ldp + colc[c]] = 0.f;
        if (inner && ok) Tg[gn * a.ldt + colc[c]] = v;
        else if (valid && ok) atomic_add(Tg + gn * a.ldt + colc[c], v);
      }
    }
}

// Many problems in one persistent launch: the work list is the concatenation
// of every problem's (cell, column tile) items (item_off[q] = first item of
// problem q, item_off[nprob] = total).  Each workgroup takes one contiguous
// range of items, so a workgroup (and, through the XCD remap, an XCD) stays on
// neighbouring cells of one problem.  Per-problem arguments, including the
// recurrence scalars, are read from the device table `descs`, so a captured
// graph stays valid when the host rewrites the table between replays.
template <int P, typename T, bool CPLX, int WAVES, int OCC, int CG, int NT>
__global__ void __attribute__((amdgpu_flat_work_group_size(64 * WAVES, 64 * WAVES), amdgpu_waves_per_eu(OCC, OCC)))
cell_hx_batched_kernel(const HxArgs<T>* __restrict__ descs, const int64_t* __restrict__ item_off, const int nprob,
                       const int contiguous) {
  __shared__ RowTables<rows_padded<P>(), T> tab;
  const int64_t nitems = item_off[nprob];
  const int64_t G = gridDim.x;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t per = (nitems + G - 1) / G;
  const int64_t i0 = contiguous ? w * per : w;
  const int64_t i1 = contiguous ? ((w + 1) * per < nitems ? (w + 1) * per : nitems) : nitems;
  const int64_t stride = contiguous ? 1 : G;
  int q = 0;
  for (int64_t it = i0; it < i1; it += stride) {
    while (q + 1 < nprob && item_off[q + 1] <= it) ++q;
    const HxArgs<T> d = descs[q];
    const int64_t local = it - item_off[q];
    const int E = d.nc * d.nc * d.nc;
    cell_item<P, T, CPLX, WAVES, 2, CG, NT>(d, static_cast<int>(local % E), static_cast<int>(local / E) * NT, tab);
  }
}

// The same work list with exactly one workgroup per item (grid = number of
// items): no item loop, the problem found by one ballot over item_off (a
// binary search chained five dependent loads at the start of every item),
// which keeps the scalar registers of the loop free for the cell item.
template <int P, typename T, bool CPLX, int WAVES, int OCC, int CG, int NT>
__global__ void __attribute__((amdgpu_flat_work_group_size(64 * WAVES, 64 * WAVES), amdgpu_waves_per_eu(OCC, OCC)))
cell_hx_batched1_kernel(const HxArgs<T>* __restrict__ descs, const int64_t* __restrict__ item_off, const int nprob) {
  __shared__ RowTables<rows_padded<P>(), T> tab;
  const int it = xcd_remap(blockIdx.x, gridDim.x);
  const int lo = __builtin_amdgcn_readfirstlane(problem_of(item_off, nprob, it));
  const HxArgs<T> d = descs[lo];
  const int local = it - static_cast<int>(item_off[lo]);
  const int E = d.nc * d.nc * d.nc;
  cell_item<P, T, CPLX, WAVES, epilogue_depth<T>(), CG, NT>(d, local % E, (local / E) * NT, tab);
}

// Launch shape of a column tile of NT columns: column groups, waves per
// workgroup and waves per SIMD.  Waves per SIMD: two for real and complex
// FP64, complex FP32 and real FP32 with four column tiles per wave (one
// workgroup's epilogue overlaps the other's MFMAs), three for real FP32 with
// two column tiles per wave; complex FP64 at p = 6 (11 row tiles per wave, A
// and B fragments doubled) needs the 512 registers of one wave per SIMD.
template <int P, typename T, bool CPLX, int NT> struct Shape {
  static constexpr int CG = NT == 32 ? 1 : col_groups<P, T, CPLX>();
  static constexpr int RG = ((P + 1) * (P + 1) * (P + 1) + 15) / 16 > 24 ? 4 : 2;
  static constexpr int WAVES = RG * CG;
  static constexpr int CPW = NT / 16 / CG;
  static constexpr int OCC = (CPLX && sizeof(T) == 8) ? (P == 6 ? 1 : 2)
                                                      : ((!CPLX && sizeof(T) == 4 && CPW == 2) ? 3 : 2);
};

template <typename T>
HxArgs<T> pack_args(const HxLaunch& L) {
  HxArgs<T> a;
  a.A = static_cast<const T*>(L.A);
  a.Ai = static_cast<const T*>(L.Ai);
  a.Ab = static_cast<const bf8*>(L.Abf);
  a.vdiag = L.vdiag;
  a.Xk = static_cast<const T*>(L.Xk);
  a.Xp = static_cast<const T*>(L.Xp);
  a.Tg = static_cast<T*>(L.T);
  a.ldx = L.ldx;
  a.ldp = L.ldp;
  a.ldt = L.ldt;
  a.ncols = L.ncols;
  a.nc = L.nc;
  a.zero_prev = L.zero_prev ? 1 : 0;
  a.alpha = static_cast<T>(L.alpha);
  a.c = static_cast<T>(L.c);
  a.beta = static_cast<T>(L.beta);
  a.pair_ptr = L.pair_ptr;
  a.pair_atom = L.pair_atom;
  a.pair_re = static_cast<const T*>(L.pair_re);
  a.pair_im = static_cast<const T*>(L.pair_im);
  a.hP = static_cast<const T*>(L.hP);
  a.ldhp = L.ldhp;
  a.astride = L.astride;
  a.cells = L.cells;
  a.ncell = L.ncell;
  return a;
}

template <int P, typename T, bool CPLX, bool BF>
hipError_t launch_p(const HxLaunch& L, hipStream_t s) {
  const HxArgs<T> a = pack_args<T>(L);
  const int64_t E = static_cast<int64_t>(L.nc) * L.nc * L.nc;
  const int nt = (BF || L.nt != 32) ? kNT : 32;   // the bf16 kernel has 64-column tiles only
  const int64_t nct = (L.ncols + nt - 1) / nt;
  const int64_t nblk = (L.cells ? L.ncell : E) * nct;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  if constexpr (BF) {
    static_assert(std::is_same<T, float>::value && !CPLX, "bf16 products: real FP32 iterates");
    hipLaunchKernelGGL((cell_hx_bf16_kernel<P>), dim3(static_cast<unsigned>(nblk)), dim3(64 * bf16_waves<P>()), 0,
                       s, a);
  } else if (nt == 32) {
    using S = Shape<P, T, CPLX, 32>;
    hipLaunchKernelGGL((cell_hx_kernel<P, T, CPLX, S::WAVES, S::OCC, S::CG, 32>), dim3(static_cast<unsigned>(nblk)),
                       dim3(64 * S::WAVES), 0, s, a);
  } else {
    using S = Shape<P, T, CPLX, kNT>;
    hipLaunchKernelGGL((cell_hx_kernel<P, T, CPLX, S::WAVES, S::OCC, S::CG, kNT>),
                       dim3(static_cast<unsigned>(nblk)), dim3(64 * S::WAVES), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T, bool CPLX, bool BF>
hipError_t launch_t(const HxLaunch& L, hipStream_t s) {
  switch (L.p) {
    case 2: return launch_p<2, T, CPLX, BF>(L, s);
    case 3: return launch_p<3, T, CPLX, BF>(L, s);
    case 4: return launch_p<4, T, CPLX, BF>(L, s);
    case 5: return launch_p<5, T, CPLX, BF>(L, s);
    case 6: return launch_p<6, T, CPLX, BF>(L, s);
    case 7: return launch_p<7, T, CPLX, BF>(L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <int P, typename T, bool CPLX, int NT>
hipError_t launch_batched_shape(const HxBatch& b, hipStream_t s) {
  using S = Shape<P, T, CPLX, NT>;
  if (b.one_per_item)
    hipLaunchKernelGGL((cell_hx_batched1_kernel<P, T, CPLX, S::WAVES, S::OCC, S::CG, NT>), dim3(b.grid),
                       dim3(64 * S::WAVES), 0, s, static_cast<const HxArgs<T>*>(b.descs), b.item_off, b.nprob);
  else
    hipLaunchKernelGGL((cell_hx_batched_kernel<P, T, CPLX, S::WAVES, S::OCC, S::CG, NT>), dim3(b.grid),
                       dim3(64 * S::WAVES), 0, s, static_cast<const HxArgs<T>*>(b.descs), b.item_off, b.nprob,
                       b.contiguous);
  return hipGetLastError();
}

template <int P, typename T, bool CPLX>
hipError_t launch_batched_p(const HxBatch& b, hipStream_t s) {
  if (b.grid <= 0 || b.nprob <= 0) return hipErrorInvalidValue;
  if (b.nt == 32) return launch_batched_shape<P, T, CPLX, 32>(b, s);
  if (b.nt == kNT) return launch_batched_shape<P, T, CPLX, kNT>(b, s);
  return hipErrorInvalidValue;
}

template <typename T, bool CPLX>
hipError_t launch_batched_t(const HxBatch& b, hipStream_t s) {
  switch (b.p) {
    case 2: return launch_batched_p<2, T, CPLX>(b, s);
    case 3: return launch_batched_p<3, T, CPLX>(b, s);
    case 4: return launch_batched_p<4, T, CPLX>(b, s);
    case 5: return launch_batched_p<5, T, CPLX>(b, s);
    case 6: return launch_batched_p<6, T, CPLX>(b, s);
    case 7: return launch_batched_p<7, T, CPLX>(b, s);
    default: return hipErrorInvalidValue;
  }
}


size_t hx_desc_bytes(int prec) {
  return (prec == CHFSI_F64 || prec == CHFSI_C128) ? sizeof(HxArgs<double>) : sizeof(HxArgs<float>);
}

void pack_hx_desc(const HxLaunch& L, int prec, void* out) {
  if (prec == CHFSI_F64 || prec == CHFSI_C128) {
    HxArgs<double> a = pack_args<double>(L);
    std::memcpy(out, &a, sizeof(a));
  } else {
    HxArgs<float> a = pack_args<float>(L);
    std::memcpy(out, &a, sizeof(a));
  }
}

hipError_t launch_cell_hx_batched(const HxBatch& b, int prec, hipStream_t s) {
  if (b.p < kMinOrder || b.p > kMaxOrder) return hipErrorInvalidValue;
  switch (prec) {
    case CHFSI_F64: return launch_batched_t<double, false>(b, s);
    case CHFSI_F32: return launch_batched_t<float, false>(b, s);
    case CHFSI_C128: return launch_batched_t<double, true>(b, s);
    case CHFSI_C64: return launch_batched_t<float, true>(b, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cell_hx(const HxLaunch& L, int prec, hipStream_t s) {
  if (L.p < kMinOrder || L.p > kMaxOrder) return hipErrorInvalidValue;
  switch (prec) {
    case CHFSI_F64: return launch_t<double, false, false>(L, s);
    case CHFSI_F32: return launch_t<float, false, false>(L, s);
    case CHFSI_BF16:
      if (L.cplx || L.Abf == nullptr) return hipErrorInvalidValue;
      return launch_t<float, false, true>(L, s);
    case CHFSI_C128: return launch_t<double, true, false>(L, s);
    case CHFSI_C64: return launch_t<float, true, false>(L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace chfsi
