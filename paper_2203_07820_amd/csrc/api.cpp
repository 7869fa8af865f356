// Host driver of libchfsi: the C ABI of include/chfsi.h.
//
// The eigensolver is DFT-FE 1.0's Chebyshev filtered eigensolver (Section
// 3.1 and Algorithm 2) at a fixed potential:
//   bound b (Lanczos), then per pass: Chebyshev filter of every column block
//   (cell-wise H~.X of Section 4.3), RRGEP-O / Cholesky / RRGEP-ST-O
//   (X <- X L^-H), RRGEP-P (H^ = X^H H~ X), RRGEP-D (dense eigensolve of the
//   N x N projected matrix) and RRGEP-ST (X <- X Q').
// The O(MN) and O(MN^2) work runs in the kernels of kernels_hx.hip and
// kernels_dense.hip.  The O(N^3) dense factorisations of the N x N matrices
// (Cholesky, triangular inverse, symmetric eigensolve) call rocSOLVER on the
// device, as the paper calls ScaLAPACK/ELPA for RRGEP-D.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <map>
#include <sstream>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "context.h"

using namespace chfsi;

thread_local std::string chfsi_host::g_create_err;

namespace {

template <typename T>
int upload(chfsi_op* op, const std::vector<T>& v, T** out) {
  *out = nullptr;
  if (v.empty()) return 0;
  void* p = nullptr;
  if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess)
    return fail(op->ctx, CHFSI_ENOMEM, "hipMalloc of operator table failed");
  op->allocs.push_back(p);
  HIP_TRY(op->ctx, hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<T*>(p);
  return 0;
}

int upload_f32(chfsi_op* op, const std::vector<double>& v, void** out) {
  std::vector<float> f(v.size());
  for (size_t i = 0; i < v.size(); ++i) f[i] = static_cast<float>(v[i]);
  float* p = nullptr;
  CHECK(upload(op, f, &p));
  *out = p;
  return 0;
}

// Colour classes of the cells for deterministic assembly.  Along each axis
// the cells of the periodic mesh form a cycle; they take colours 0, 1, 0,
// 1, ... and, when the number of cells per side is odd, the last cell colour
// 2, so that neighbouring cells never share a colour.  A class is a triple
// of axis colours (8 classes for an even side, 27 for an odd one); two
// cells of one class are not neighbours along any axis and so share no
// node, which the construction checks by marking the nodes of each class.
int build_colours(chfsi_op* op) {
  if (op->colour_cells) return 0;
  const HostTables& t = op->t;
  const int nc = t.ncell, p = t.p, n = nc * p;
  if (nc < 2)
    return fail(op->ctx, CHFSI_EINVAL,
                "deterministic assembly needs at least 2 cells per side (a single cell shares nodes with its "
                "own periodic images)");
  const int K = (nc % 2) ? 3 : 2;
  auto colour = [&](int i) { return (nc % 2 && i == nc - 1) ? 2 : i % 2; };
  std::vector<std::vector<int32_t>> cls(K * K * K);
  for (int cz = 0; cz < nc; ++cz)
    for (int cy = 0; cy < nc; ++cy)
      for (int cx = 0; cx < nc; ++cx)
        cls[colour(cx) + K * (colour(cy) + K * colour(cz))].push_back(cx + nc * (cy + nc * cz));
  std::vector<int32_t> mark(static_cast<size_t>(n) * n * n, -1);
  std::vector<int32_t> flat;
  std::vector<int> off{0};
  for (int k = 0; k < K * K * K; ++k) {
    if (cls[k].empty()) continue;
    for (const int32_t cell : cls[k]) {
      const int cx = cell % nc, cy = (cell / nc) % nc, cz = cell / (nc * nc);
      for (int lc = 0; lc <= p; ++lc)
        for (int lb = 0; lb <= p; ++lb)
          for (int la = 0; la <= p; ++la) {
            const int gx = (cx * p + la) % n, gy = (cy * p + lb) % n, gz = (cz * p + lc) % n;
            int32_t& m = mark[gx + static_cast<size_t>(n) * (gy + static_cast<size_t>(n) * gz)];
            if (m == k) return fail(op->ctx, CHFSI_EINVAL, "internal error: a colour class shares a node");
            m = k;
          }
    }
    flat.insert(flat.end(), cls[k].begin(), cls[k].end());
    off.push_back(static_cast<int>(flat.size()));
  }
  int32_t* d = nullptr;
  CHECK(upload(op, flat, &d));
  op->colour_cells = d;
  op->colour_off = off;
  return 0;
}

// One H~.X launch over all cells, or, with deterministic assembly, one per
// colour class in a fixed order: inside a class every node receives at most
// one contribution, so each node's sum is formed in the class order
// whatever the order in which the workgroups run.
int launch_hx_cells(chfsi_op* op, const HxLaunch& L, int prec) {
  chfsi_ctx* ctx = op->ctx;
  if (!ctx->deterministic) {
    HIP_TRY(ctx, launch_cell_hx(L, prec, ctx->stream));
    return 0;
  }
  if (!op->colour_cells) {
    if (op->t.ncell < 2) CHECK(build_colours(op));   // fails with the reason
    return fail(ctx, CHFSI_EINVAL, "colour classes of the operator are not built");
  }
  for (size_t k = 0; k + 1 < op->colour_off.size(); ++k) {
    HxLaunch Lk = L;
    Lk.cells = op->colour_cells + op->colour_off[k];
    Lk.ncell = op->colour_off[k + 1] - op->colour_off[k];
    HIP_TRY(ctx, launch_cell_hx(Lk, prec, ctx->stream));
  }
  return 0;
}

bool prec_valid_for(const chfsi_op* op, int prec) {
  if (op->t.cplx) return prec == CHFSI_C128 || prec == CHFSI_C64;
  // per-cell matrices exist in FP64 and FP32 only
  return prec == CHFSI_F64 || prec == CHFSI_F32 || (prec == CHFSI_BF16 && op->astride == 0);
}

size_t prec_bytes(int prec) {
  switch (prec) {
    case CHFSI_F64: return 8;
    case CHFSI_F32: case CHFSI_BF16: return 4;
    case CHFSI_C128: return 16;
    case CHFSI_C64: return 8;
    default: return 0;
  }
}

// storage precision used for a given arithmetic precision
int storage_of(int prec) { return prec == CHFSI_BF16 ? CHFSI_F32 : prec; }
bool is_single(int prec) { return prec == CHFSI_F32 || prec == CHFSI_BF16 || prec == CHFSI_C64; }

// P = h * C^H Xk for the projectors of op (node-level lists, deterministic
// two-phase sum) into hP (natoms*4 x ldhp, real view), using `part` as the
// chunk partials (nchunks*4 x ldhp).
NlLaunch make_nl(const chfsi_op* op, const void* Xk, int64_t ldx, int64_t ncols, void* part, void* hP,
                 int64_t ldhp) {
  const HostTables& t = op->t;
  NlLaunch nl;
  nl.natoms = t.natoms;
  nl.cplx = t.cplx;
  nl.ncols = static_cast<int>(ncols);
  nl.atom_ptr = op->atom_ptr;
  nl.atom_node = op->atom_node;
  nl.atom_val = op->atom_val;
  nl.chunk_atom = op->chunk_atom;
  nl.chunk_begin = op->chunk_begin;
  nl.nchunks = op->nchunks;
  nl.atom_chunk_ptr = op->atom_chunk_ptr;
  nl.hcoef = op->hcoef;
  nl.X = Xk;
  nl.ldx = ldx;
  nl.partial = part;
  nl.hP = hP;
  nl.ldhp = ldhp;
  return nl;
}

int nl_project(chfsi_op* op, int prec, const void* Xk, int64_t ldx, int64_t ncols, void* part, void* hP,
               int64_t ldhp) {
  chfsi_ctx* ctx = op->ctx;
  const NlLaunch nl = make_nl(op, Xk, ldx, ncols, part, hP, ldhp);
  HIP_TRY(ctx, launch_nl_project(nl, prec, ctx->stream));
  return 0;
}

int64_t hp_ld(const chfsi_op* op, int64_t ncols) { return (ncols * (op->t.cplx ? 2 : 1) + 63) / 64 * 64; }

// Kernel arguments of one step T += alpha (H~ Xk - c Xk) - beta Xp (logical lds).
HxLaunch make_hx(const chfsi_op* op, int prec, const void* Xk, int64_t ldx, const void* Xp, int64_t ldp, void* T,
                 int64_t ldt, int64_t ncols, double alpha, double c, double beta, bool zero_prev, const void* hP,
                 int64_t ldhp) {
  const HostTables& t = op->t;
  const int cf = t.cplx ? 2 : 1;
  const bool single = is_single(prec);
  HxLaunch L;
  L.p = t.p;
  L.nc = t.ncell;
  L.ncols = static_cast<int>(ncols * cf);
  L.cplx = t.cplx;
  // a block of at most 32 real columns takes the 32-column work item (half
  // the padding of a 64-column one)
  L.nt = (prec != CHFSI_BF16 && L.ncols <= 32) ? 32 : 64;
  L.A = single ? op->A32 : op->A64;
  L.astride = op->astride;
  L.Ai = single ? op->Ai32 : op->Ai64;
  L.vdiag = op->vdiag;
  L.Xk = Xk;
  L.ldx = ldx * cf;
  L.Xp = Xp;
  L.ldp = ldp * cf;
  L.T = T;
  L.ldt = ldt * cf;
  L.zero_prev = zero_prev;
  L.alpha = alpha;
  L.c = c;
  L.beta = beta;
  L.pair_ptr = t.has_proj ? op->pair_ptr : nullptr;
  L.pair_atom = op->pair_atom;
  L.pair_re = single ? op->pair_re32 : op->pair_re64;
  L.pair_im = single ? op->pair_im32 : op->pair_im64;
  L.hP = hP;
  L.ldhp = ldhp;
  L.Abf = op->Abf;
  L.ncu = op->ctx->ncu;
  return L;
}

// algorithmic flops of one step over ncols logical columns (padding excluded)
double hx_flops(const chfsi_op* op, int64_t ncols) {
  const HostTables& t = op->t;
  const double cfl = t.cplx ? 4.0 : 1.0;
  double fl = 2.0 * t.mcell * static_cast<double>(t.mcell) * static_cast<double>(ncols) * t.E * cfl;
  if (t.has_proj) fl += 2.0 * 2.0 * t.mcell * 4.0 * static_cast<double>(ncols) * op->npairs * cfl;
  return fl;
}

// the part of hx_flops that the cell kernel itself does: the cell products
// and C (h P) per (cell, atom) pair, without the projection P = C^H X, which
// the nonlocal kernels do before it
double cell_kernel_flops(const chfsi_op* op, int64_t ncols) {
  const HostTables& t = op->t;
  const double cfl = t.cplx ? 4.0 : 1.0;
  double fl = 2.0 * t.mcell * static_cast<double>(t.mcell) * static_cast<double>(ncols) * t.E * cfl;
  if (t.has_proj) fl += 2.0 * t.mcell * 4.0 * static_cast<double>(ncols) * op->npairs * cfl;
  return fl;
}

// Y = alpha (H~ Xk - c Xk) - beta Xp  accumulated into T (which must hold 0
// on entry).  Xk, Xp, T are in the storage type of prec, logical ld.
int hx_step(chfsi_op* op, int prec, const void* Xk, int64_t ldx, const void* Xp, int64_t ldp, void* T,
            int64_t ldt, int64_t ncols, double alpha, double c, double beta, bool zero_prev) {
  chfsi_ctx* ctx = op->ctx;
  const HostTables& t = op->t;
  const bool single = is_single(prec);
  void* hP = nullptr;
  int64_t ldhp = 0;
  if (t.has_proj) {
    ldhp = hp_ld(op, ncols);
    const size_t eb = single ? 4 : 8;
    void* part = nullptr;
    CHECK(ws_get(ctx, WS_NLPART, static_cast<size_t>(op->nchunks) * 4 * ldhp * eb, &part));
    CHECK(ws_get(ctx, WS_HP, static_cast<size_t>(t.natoms) * 4 * ldhp * eb, &hP));
    CHECK(nl_project(op, prec, Xk, ldx, ncols, part, hP, ldhp));
  }
  HxLaunch L = make_hx(op, prec, Xk, ldx, Xp, ldp, T, ldt, ncols, alpha, c, beta, zero_prev, hP, ldhp);
  const int kp = prec;
  if (ctx->deterministic) CHECK(build_colours(op));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timing) {
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
  }
  CHECK(launch_hx_cells(op, L, kp));
  if (ctx->timing) {
    HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    ctx->pending.emplace_back(e0, e1);
    ctx->pending_flops.push_back(cell_kernel_flops(op, ncols));
  }
  return 0;
}

// Scaled Chebyshev coefficients (Section 3.1 filter; the three-term recurrence
// rescaled each step): step 1 Y = a1 (H~X - cX); step i >= 2
// Z = a_i (H~Y - cY) - b_i X.
void cheb_coeffs(int m, double a, double b, double aL, double* c, std::vector<double>& al,
                 std::vector<double>& be) {
  const double e = (b - a) / 2.0;
  *c = (b + a) / 2.0;
  const double s1 = e / (aL - *c);
  double s = s1;
  al.assign(m, 0.0);
  be.assign(m, 0.0);
  al[0] = s1 / e;
  for (int i = 1; i < m; ++i) {
    const double sn = 1.0 / (2.0 / s1 - s);
    al[i] = 2.0 * sn / e;
    be[i] = s * sn;
    s = sn;
  }
}

// Filter one block already converted into R0 (storage of prec, ld = ncols).
// Returns the index of the buffer holding the result.
// Filters the block held in R[0] (ncols columns, leading dimensions ldr[i])
// with the buffers R[1..3]; the result is in R[*out_idx].
int filter_block(chfsi_op* op, int prec, void* const R[4], int64_t ncols, const int64_t ldr[4], int m, double a,
                 double b, double aL, int* out_idx) {
  chfsi_ctx* ctx = op->ctx;
  const int cf = op->t.cplx ? 2 : 1;
  const int64_t M = op->t.M;
  double c;
  std::vector<double> al, be;
  cheb_coeffs(m, a, b, aL, &c, al, be);
  const int sp = storage_of(prec);
  for (int i = 1; i < 4; ++i) HIP_TRY(ctx, launch_fill(R[i], M, ncols * cf, ldr[i] * cf, sp, ctx->stream));
  CHECK(hx_step(op, prec, R[0], ldr[0], nullptr, ldr[0], R[1], ldr[1], ncols, al[0], c, 0.0, false));
  for (int i = 2; i <= m; ++i) {
    const int k = (i - 1) % 4, p = (i - 2) % 4, t = i % 4;
    CHECK(hx_step(op, prec, R[k], ldr[k], R[p], ldr[p], R[t], ldr[t], ncols, al[i - 1], c, be[i - 1], true));
  }
  *out_idx = m % 4;
  return 0;
}

int do_filter(chfsi_op* op, void* X, int64_t ncols, int64_t ld, int m, double a, double b, double aL, int prec,
              int64_t block) {
  chfsi_ctx* ctx = op->ctx;
  const HostTables& t = op->t;
  const int cf = t.cplx ? 2 : 1;
  const int xprec = t.cplx ? CHFSI_C128 : CHFSI_F64;
  const int sp = storage_of(prec);
  if (block <= 0 || block > ncols) block = ncols;
  const size_t eb = prec_bytes(sp);
  // the work buffers' rows are padded to a multiple of 4 columns (16-byte
  // aligned rows for the bf16 kernel's block loads)
  const int64_t ldmax = (block + 3) / 4 * 4;
  void* R[4];
  for (int i = 0; i < 4; ++i) CHECK(ws_get(ctx, WS_R0 + i, static_cast<size_t>(t.M) * ldmax * eb, &R[i]));
  // in the block's own storage type the caller's block itself is the first
  // buffer of the rotation (no copy in; the owners clear its rows at step 2
  // for reuse as a target, and the result, unless it lands there, is copied
  // back over it)
  const bool in_place = sp == xprec;
  for (int64_t c0 = 0; c0 < ncols; c0 += block) {
    const int64_t nb = std::min<int64_t>(block, ncols - c0);
    const int64_t ldw = (nb + 3) / 4 * 4;
    double* Xb = static_cast<double*>(X) + c0 * cf;
    void* Rb[4] = {R[0], R[1], R[2], R[3]};
    int64_t ldr[4] = {ldw, ldw, ldw, ldw};
    if (in_place) {
      Rb[0] = Xb;
      ldr[0] = ld;
    } else {
      HIP_TRY(ctx, launch_convert(R[0], ldw * cf, sp, Xb, ld * cf, xprec, t.M, nb * cf, ctx->stream));
    }
    int idx = 0;
    CHECK(filter_block(op, prec, Rb, nb, ldr, m, a, b, aL, &idx));
    if (!(in_place && idx == 0))
      HIP_TRY(ctx, launch_convert(Xb, ld * cf, xprec, Rb[idx], ldr[idx] * cf, sp, t.M, nb * cf, ctx->stream));
  }
  return 0;
}

// ---- dense helpers ----------------------------------------------------------

// S (N x N, column-major; complex interleaved) = X^H Y over real views, into
// *S_out, or into the context's workspace when *S_out is null on entry.
int gram(chfsi_op* op, const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t N, double** S_out) {
  chfsi_ctx* ctx = op->ctx;
  const int cf = op->t.cplx ? 2 : 1;
  const int n = static_cast<int>(N * cf);
  void *part, *G, *S = *S_out;
  CHECK(ws_get(ctx, WS_GPART, gram_partial_bytes(op->t.M, n, std::max(ldx, ldy) * cf), &part));
  CHECK(ws_get(ctx, WS_G, static_cast<size_t>(n) * n * 8, &G));
  if (!S) CHECK(ws_get(ctx, WS_S, static_cast<size_t>(N) * N * 8 * cf, &S));
  HIP_TRY(ctx, launch_gram(X, ldx * cf, Y, ldy * cf, op->t.M, n, static_cast<double*>(part),
                           static_cast<double*>(G), n, ctx->stream));
  if (op->t.cplx)
    HIP_TRY(ctx, launch_gram_combine_complex(static_cast<double*>(G), n, static_cast<double*>(S),
                                             static_cast<int>(N), ctx->stream));
  else
    HIP_TRY(ctx, launch_sym_from_lower(static_cast<double*>(G), n, static_cast<double*>(S), n, ctx->stream));
  *S_out = static_cast<double*>(S);
  return 0;
}

int read_info(chfsi_ctx* ctx, rocblas_int* dinfo, int* info) {
  rocblas_int h = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&h, dinfo, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *info = h;
  return 0;
}

// CholGS: Xout = X L^-H with S = X^H X = L L^H.  Xout may not alias X.  On
// CHFSI_ECHOL, *bad_col (nullable) receives the first column that is a
// combination of the earlier ones to working precision.
int cholgs(chfsi_op* op, const double* X, int64_t ldx, double* Xout, int64_t ldo, int64_t N, double* L_host,
           int64_t* bad_col = nullptr) {
  chfsi_ctx* ctx = op->ctx;
  const bool cplx = op->t.cplx;
  const int cf = cplx ? 2 : 1;
  double* S = nullptr;
  CHECK(gram(op, X, ldx, X, ldx, N, &S));
  void* dinfo;
  CHECK(ws_get(ctx, WS_INFO, 64, &dinfo));
  const rocblas_int n = static_cast<rocblas_int>(N);
  int info = 0;
  // small blocks: factor and inverse in one workgroup (the factor itself is
  // not kept, so a caller asking for L takes the library route)
  const bool small = N <= kSmallMaxN && L_host == nullptr;
  if (small) {
    SmallBatch sb;
    sb.mat0 = S;
    sb.n0 = static_cast<int>(N);
    sb.info = static_cast<int*>(dinfo);
    HIP_TRY(ctx, launch_small_cholinv(sb, 1, cplx, ctx->stream));
  } else if (cplx) {
    RB_TRY(ctx, rocsolver_zpotrf(ctx->blas, rocblas_fill_lower, n, reinterpret_cast<rocblas_double_complex*>(S), n,
                                 static_cast<rocblas_int*>(dinfo)));
  } else {
    RB_TRY(ctx, rocsolver_dpotrf(ctx->blas, rocblas_fill_lower, n, S, n, static_cast<rocblas_int*>(dinfo)));
  }
  CHECK(read_info(ctx, static_cast<rocblas_int*>(dinfo), &info));
  if (info != 0) {
    if (bad_col) *bad_col = info - 1;   // the leading minor of order info fails
    return fail(ctx, CHFSI_ECHOL, "overlap matrix is not positive definite (leading minor " + std::to_string(info) +
                                      ")");
  }
  if (L_host) {
    std::vector<double> Lcm(static_cast<size_t>(N) * N * cf);
    HIP_TRY(ctx, hipMemcpyAsync(Lcm.data(), S, Lcm.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t i = 0; i < N; ++i)
      for (int64_t j = 0; j < N; ++j)
        for (int q = 0; q < cf; ++q)
          L_host[(i * N + j) * cf + q] = (i >= j) ? Lcm[(i + j * N) * cf + q] : 0.0;
  }
  if (!small) {
    if (cplx)
      RB_TRY(ctx, rocsolver_ztrtri(ctx->blas, rocblas_fill_lower, rocblas_diagonal_non_unit, n,
                                   reinterpret_cast<rocblas_double_complex*>(S), n, static_cast<rocblas_int*>(dinfo)));
    else
      RB_TRY(ctx, rocsolver_dtrtri(ctx->blas, rocblas_fill_lower, rocblas_diagonal_non_unit, n, S, n,
                                   static_cast<rocblas_int*>(dinfo)));
    CHECK(read_info(ctx, static_cast<rocblas_int*>(dinfo), &info));
    if (info != 0) return fail(ctx, CHFSI_ECHOL, "Cholesky factor is singular");
  }
  // Z = L^-H (upper triangular), as a real-view matrix
  const double* Z = nullptr;
  int64_t ldz = 0;
  if (cplx) {
    void* Z2;
    CHECK(ws_get(ctx, WS_Z2, static_cast<size_t>(N) * N * 4 * 8, &Z2));
    HIP_TRY(ctx, launch_expand_complex(S, n, n, 1, static_cast<double*>(Z2), ctx->stream));
    Z = static_cast<double*>(Z2);
    ldz = 2 * N;
  } else {
    HIP_TRY(ctx, launch_zero_strict_lower(S, n, N, ctx->stream));
    Z = S;
    ldz = N;
  }
  HIP_TRY(ctx, launch_rotate(X, ldx * cf, Z, ldz, Xout, ldo * cf, op->t.M, static_cast<int>(N * cf),
                             static_cast<int>(N * cf), true, ctx->stream));
  return 0;
}

// Rayleigh-Ritz on orthonormal X.  Writes Psi to Psi_out (may not alias X),
// theta (host), resid (host, nullable).  W is scratch.
int rayleigh_ritz(chfsi_op* op, const double* X, int64_t ldx, double* Psi, int64_t ldpsi, int64_t N,
                  double* theta, double* resid) {
  chfsi_ctx* ctx = op->ctx;
  const HostTables& t = op->t;
  const bool cplx = t.cplx;
  const int cf = cplx ? 2 : 1;
  const int prec = cplx ? CHFSI_C128 : CHFSI_F64;
  void *W, *HPsi;
  CHECK(ws_get(ctx, WS_W, static_cast<size_t>(t.M) * N * 8 * cf, &W));
  HIP_TRY(ctx, launch_fill(W, t.M, N * cf, N * cf, prec, ctx->stream));
  CHECK(hx_step(op, prec, X, ldx, nullptr, 0, W, N, N, 1.0, 0.0, 0.0, false));
  double* Hh = nullptr;
  CHECK(gram(op, X, ldx, static_cast<double*>(W), N, N, &Hh));
  void *dinfo, *eig;
  CHECK(ws_get(ctx, WS_INFO, 64, &dinfo));
  CHECK(ws_get(ctx, WS_EIG, static_cast<size_t>(N) * 2 * 8, &eig));
  double* D = static_cast<double*>(eig);
  double* Ework = D + N;
  const rocblas_int n = static_cast<rocblas_int>(N);
  // small blocks: Jacobi in one workgroup; its convergence flag is read with
  // the results at the end instead of through a synchronisation here
  const bool small = N <= kSmallMaxN;
  int info = 0;
  if (small) {
    SmallBatch sb;
    sb.mat0 = Hh;
    sb.n0 = static_cast<int>(N);
    sb.ev0 = D;
    sb.info = static_cast<int*>(dinfo);
    HIP_TRY(ctx, launch_small_eigh(sb, 1, cplx, ctx->stream));
  } else {
    if (cplx)
      RB_TRY(ctx, rocsolver_zheevd(ctx->blas, rocblas_evect_original, rocblas_fill_lower, n,
                                   reinterpret_cast<rocblas_double_complex*>(Hh), n, D, Ework,
                                   static_cast<rocblas_int*>(dinfo)));
    else
      RB_TRY(ctx, rocsolver_dsyevd(ctx->blas, rocblas_evect_original, rocblas_fill_lower, n, Hh, n, D, Ework,
                                   static_cast<rocblas_int*>(dinfo)));
    CHECK(read_info(ctx, static_cast<rocblas_int*>(dinfo), &info));
    if (info != 0) return fail(ctx, CHFSI_EHIP, "projected eigensolve did not converge");
  }
  const double* Z = nullptr;
  int64_t ldz = 0;
  void* Zb;
  if (cplx) {
    CHECK(ws_get(ctx, WS_Z2, static_cast<size_t>(N) * N * 4 * 8, &Zb));
    HIP_TRY(ctx, launch_expand_complex(Hh, n, n, 2, static_cast<double*>(Zb), ctx->stream));
    ldz = 2 * N;
  } else {
    CHECK(ws_get(ctx, WS_Z, static_cast<size_t>(N) * N * 8, &Zb));
    HIP_TRY(ctx, launch_transpose(Hh, static_cast<double*>(Zb), n, ctx->stream));
    ldz = N;
  }
  Z = static_cast<double*>(Zb);
  HIP_TRY(ctx, launch_rotate(X, ldx * cf, Z, ldz, Psi, ldpsi * cf, t.M, static_cast<int>(N * cf),
                             static_cast<int>(N * cf), false, ctx->stream));
  if (resid) {
    CHECK(ws_get(ctx, WS_HPSI, static_cast<size_t>(t.M) * N * 8 * cf, &HPsi));
    HIP_TRY(ctx, launch_rotate(static_cast<double*>(W), N * cf, Z, ldz, static_cast<double*>(HPsi), N * cf, t.M,
                               static_cast<int>(N * cf), static_cast<int>(N * cf), false, ctx->stream));
    void* rp;
    CHECK(ws_get(ctx, WS_RPART, resid_partial_count(t.M, static_cast<int>(N)) * 8, &rp));
    int nch = 0;
    HIP_TRY(ctx, launch_resid(static_cast<double*>(HPsi), N, Psi, ldpsi, D, t.M, static_cast<int>(N), cplx,
                              static_cast<double*>(rp), &nch, ctx->stream));
    std::vector<double> hp(static_cast<size_t>(nch) * N);
    HIP_TRY(ctx, hipMemcpyAsync(hp.data(), rp, hp.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(theta, D, N * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (small) HIP_TRY(ctx, hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (info != 0) return fail(ctx, CHFSI_EHIP, "projected eigensolve did not converge");
    for (int64_t j = 0; j < N; ++j) {
      double s = 0.0;
      for (int c = 0; c < nch; ++c) s += hp[static_cast<size_t>(c) * N + j];
      resid[j] = std::sqrt(s);
    }
  } else {
    HIP_TRY(ctx, hipMemcpyAsync(theta, D, N * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (small) HIP_TRY(ctx, hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (info != 0) return fail(ctx, CHFSI_EHIP, "projected eigensolve did not converge");
  }
  return 0;
}

// Rayleigh-Ritz through the generalised eigenproblem with spectrum splitting
// (Algorithm 2).  X (M x N, ldx; complex interleaved for a complex operator)
// holds the filtered block on entry and Psi_o = X L^-H on exit; Pfr (M x nfr,
// ldfr) receives the nfr highest Ritz vectors X Q_fr; theta (host, N) all
// generalised eigenvalues.  mixed: S off-diagonal 128-column blocks and H^
// outside its fr-fr block from FP32 copies in FP32 arithmetic, Psi_o =
// FP32[X L^-H without diagonal] + FP64[X diag(L^-H)].  Complex data goes
// through the real views (2N real columns) of the Gram and rotation kernels.
int rrgep_split(chfsi_op* op, double* X, int64_t ldx, int64_t N, int nfr, bool mixed, double* theta, double* Pfr,
                int64_t ldfr) {
  chfsi_ctx* ctx = op->ctx;
  const HostTables& t = op->t;
  const bool cplx = t.cplx;
  const int cf = cplx ? 2 : 1;
  const int64_t M = t.M, nr = N * cf, ldxr = ldx * cf;
  const int n = static_cast<int>(N), nrr = static_cast<int>(nr);
  const int prec = cplx ? CHFSI_C128 : CHFSI_F64;
  hipStream_t st = ctx->stream;
  void *W, *part, *G, *S, *Hh, *Zb, *dinfo, *eig;
  CHECK(ws_get(ctx, WS_W, static_cast<size_t>(M) * nr * 8, &W));
  // the partial buffer serves the full Gram and the 128-wide and fr-wide ones
  const int64_t ldm = std::max<int64_t>(ldxr, nr);
  const size_t pbytes = std::max({gram_partial_bytes(M, nrr, ldm), gram_partial_bytes(M, std::min(n, 128) * cf, ldm),
                                  gram_partial_bytes(M, nfr * cf, ldm)});
  CHECK(ws_get(ctx, WS_GPART, pbytes, &part));
  CHECK(ws_get(ctx, WS_RR_G, static_cast<size_t>(nr) * nr * 8 + static_cast<size_t>(nr) * 8, &G));
  CHECK(ws_get(ctx, WS_RR_S, static_cast<size_t>(N) * N * 8 * cf, &S));
  CHECK(ws_get(ctx, WS_RR_H, static_cast<size_t>(N) * N * 8 * cf, &Hh));
  CHECK(ws_get(ctx, WS_RR_Z, static_cast<size_t>(nr) * nr * 8, &Zb));
  CHECK(ws_get(ctx, WS_INFO, 64, &dinfo));
  CHECK(ws_get(ctx, WS_EIG, static_cast<size_t>(N) * 3 * 8, &eig));
  double* Gd = static_cast<double*>(G);
  double* Sd = static_cast<double*>(S);
  double* Hd = static_cast<double*>(Hh);
  double* Zd = static_cast<double*>(Zb);
  double* D = static_cast<double*>(eig);
  double* Ework = D + N;
  double* Wd = static_cast<double*>(W);
  double* partd = static_cast<double*>(part);
  auto hermitian = [&](double* dst) -> int {   // dst (N x N, column-major) from the lower real-view Gram
    if (cplx) HIP_TRY(ctx, launch_gram_combine_complex(Gd, nr, dst, n, st));
    else HIP_TRY(ctx, launch_sym_from_lower(Gd, nr, dst, n, st));
    return 0;
  };
  // RRGEP-P needs W = H~ X
  HIP_TRY(ctx, launch_fill(W, M, nr, nr, prec, st));
  CHECK(hx_step(op, prec, X, ldx, nullptr, 0, W, N, N, 1.0, 0.0, 0.0, false));
  float *X32 = nullptr, *W32 = nullptr;
  if (mixed) {
    void *a, *b;
    CHECK(ws_get(ctx, WS_X32, static_cast<size_t>(M) * nr * 4, &a));
    CHECK(ws_get(ctx, WS_W32, static_cast<size_t>(M) * nr * 4, &b));
    X32 = static_cast<float*>(a);
    W32 = static_cast<float*>(b);
    HIP_TRY(ctx, launch_convert(X32, nr, CHFSI_F32, X, ldxr, CHFSI_F64, M, nr, st));
    HIP_TRY(ctx, launch_convert(W32, nr, CHFSI_F32, W, nr, CHFSI_F64, M, nr, st));
  }
  // RRGEP-O: lower tiles of S; with mixed, FP32 everywhere, then the
  // diagonal blocks of 128 columns again in FP64
  if (mixed) {
    HIP_TRY(ctx, launch_gram(X32, nr, X32, nr, M, nrr, partd, Gd, nr, st));
    for (int64_t c0 = 0; c0 < N; c0 += 128) {
      const int nb = static_cast<int>(std::min<int64_t>(128, N - c0)) * cf;
      const int64_t o = c0 * cf;
      HIP_TRY(ctx, launch_gram(X + o, ldxr, X + o, ldxr, M, nb, partd, Gd + o * nr + o, nr, st, o, o));
    }
  } else {
    HIP_TRY(ctx, launch_gram(X, ldxr, X, ldxr, M, nrr, partd, Gd, nr, st));
  }
  CHECK(hermitian(Sd));
  // RRGEP-P: H^ = X^H W; with mixed, FP32 except the fr-fr block
  const int64_t f0 = N - nfr, fo = f0 * cf;
  if (mixed) {
    HIP_TRY(ctx, launch_gram(X32, nr, W32, nr, M, nrr, partd, Gd, nr, st));
    HIP_TRY(ctx, launch_gram(X + fo, ldxr, Wd + fo, nr, M, nfr * cf, partd, Gd + fo * nr + fo, nr, st, fo, fo));
  } else {
    HIP_TRY(ctx, launch_gram(X, ldxr, Wd, nr, M, nrr, partd, Gd, nr, st));
  }
  CHECK(hermitian(Hd));
  // RRGEP-D: S = L L^H, H' = L^-1 H^ L^-H, eigenpairs, Q_fr = L^-H Q'_fr
  const rocblas_int rn = static_cast<rocblas_int>(N), rf = static_cast<rocblas_int>(nfr);
  rocblas_int* di = static_cast<rocblas_int*>(dinfo);
  auto zc = [](double* p) { return reinterpret_cast<rocblas_double_complex*>(p); };
  if (cplx) RB_TRY(ctx, rocsolver_zpotrf(ctx->blas, rocblas_fill_lower, rn, zc(Sd), rn, di));
  else RB_TRY(ctx, rocsolver_dpotrf(ctx->blas, rocblas_fill_lower, rn, Sd, rn, di));
  int info = 0;
  CHECK(read_info(ctx, di, &info));
  if (info != 0)
    return fail(ctx, CHFSI_ECHOL, "overlap matrix is not positive definite (leading minor " + std::to_string(info) +
                                      ")");
  const double one = 1.0;
  const rocblas_double_complex zone(1.0, 0.0);
  if (cplx) {
    RB_TRY(ctx, rocblas_ztrsm(ctx->blas, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                              rocblas_diagonal_non_unit, rn, rn, &zone, zc(Sd), rn, zc(Hd), rn));
    RB_TRY(ctx, rocblas_ztrsm(ctx->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_conjugate_transpose,
                              rocblas_diagonal_non_unit, rn, rn, &zone, zc(Sd), rn, zc(Hd), rn));
    RB_TRY(ctx, rocsolver_zheevd(ctx->blas, rocblas_evect_original, rocblas_fill_lower, rn, zc(Hd), rn, D, Ework, di));
  } else {
    RB_TRY(ctx, rocblas_dtrsm(ctx->blas, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                              rocblas_diagonal_non_unit, rn, rn, &one, Sd, rn, Hd, rn));
    RB_TRY(ctx, rocblas_dtrsm(ctx->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                              rocblas_diagonal_non_unit, rn, rn, &one, Sd, rn, Hd, rn));
    RB_TRY(ctx, rocsolver_dsyevd(ctx->blas, rocblas_evect_original, rocblas_fill_lower, rn, Hd, rn, D, Ework, di));
  }
  CHECK(read_info(ctx, di, &info));
  if (info != 0) return fail(ctx, CHFSI_EHIP, "projected eigensolve did not converge");
  double* Qfr = Hd + f0 * N * cf;  // column-major N x nfr
  if (cplx)
    RB_TRY(ctx, rocblas_ztrsm(ctx->blas, rocblas_side_left, rocblas_fill_lower, rocblas_operation_conjugate_transpose,
                              rocblas_diagonal_non_unit, rn, rf, &zone, zc(Sd), rn, zc(Qfr), rn));
  else
    RB_TRY(ctx, rocblas_dtrsm(ctx->blas, rocblas_side_left, rocblas_fill_lower, rocblas_operation_transpose,
                              rocblas_diagonal_non_unit, rn, rf, &one, Sd, rn, Qfr, rn));
  // RRGEP-ST-F: Psi^R_fr = X Q_fr through a row-major real-view (nr x nfr cf) Z
  if (cplx) HIP_TRY(ctx, launch_expand_complex(Qfr, n, nfr, 2, Zd, st));
  else HIP_TRY(ctx, launch_transpose_rect(Qfr, N, nfr, n, Zd, nfr, st));
  HIP_TRY(ctx, launch_rotate(X, ldxr, Zd, nfr * cf, Pfr, ldfr * cf, M, nrr, nfr * cf, false, st));
  // RRGEP-ST-O: Psi_o = X L^-H.  Real: the column-major lower L^-1 read
  // row-major is L^-T once its other triangle is cleared; complex: expanded
  // into the real-view upper block-triangular matrix
  if (cplx) RB_TRY(ctx, rocsolver_ztrtri(ctx->blas, rocblas_fill_lower, rocblas_diagonal_non_unit, rn, zc(Sd), rn, di));
  else RB_TRY(ctx, rocsolver_dtrtri(ctx->blas, rocblas_fill_lower, rocblas_diagonal_non_unit, rn, Sd, rn, di));
  CHECK(read_info(ctx, di, &info));
  if (info != 0) return fail(ctx, CHFSI_ECHOL, "Cholesky factor is singular");
  const double* Zr = Sd;
  if (cplx) {
    HIP_TRY(ctx, launch_expand_complex(Sd, n, n, 1, Zd, st));
    Zr = Zd;
  } else {
    HIP_TRY(ctx, launch_zero_strict_lower(Sd, n, N, st));
  }
  if (mixed) {
    void* c32;
    CHECK(ws_get(ctx, WS_C32, static_cast<size_t>(M) * nr * 4, &c32));
    float* Z32 = reinterpret_cast<float*>(Gd);  // nr x nr floats, then nr doubles of the diagonal
    double* dg = Gd + (nr * nr + 1) / 2;
    HIP_TRY(ctx, launch_split_diag(Zr, nr, nrr, Z32, dg, st));
    HIP_TRY(ctx, launch_rotate(X32, nr, Z32, nr, static_cast<float*>(c32), nr, M, nrr, nrr, true, st));
    HIP_TRY(ctx, launch_add_scaled_cols(static_cast<float*>(c32), nr, dg, X, ldxr, M, nrr, st));
  } else {
    void* X2;
    CHECK(ws_get(ctx, WS_X2, static_cast<size_t>(M) * nr * 8, &X2));
    HIP_TRY(ctx, launch_rotate(X, ldxr, Zr, nr, static_cast<double*>(X2), nr, M, nrr, nrr, true, st));
    HIP_TRY(ctx, launch_convert(X, ldxr, CHFSI_F64, X2, nr, CHFSI_F64, M, nr, st));
  }
  HIP_TRY(ctx, hipMemcpyAsync(theta, D, N * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  return 0;
}

// Eigenvalues of a small symmetric matrix by cyclic Jacobi rotations.
std::vector<double> small_eigvals(std::vector<double> A, int n) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double tt = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(tt * tt + 1.0), sn = tt * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = cs * akp - sn * akq;
          A[k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = cs * apk - sn * aqk;
          A[q * n + k] = sn * apk + cs * aqk;
        }
      }
  }
  std::vector<double> ev(n);
  for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
  std::sort(ev.begin(), ev.end());
  return ev;
}

int dot_host(chfsi_ctx* ctx, const double* x, const double* y, int64_t n, double* out) {
  void* part;
  CHECK(ws_get(ctx, WS_SMALL, dot_blocks() * 8, &part));
  HIP_TRY(ctx, launch_dot(x, y, n, static_cast<double*>(part), ctx->stream));
  std::vector<double> h(dot_blocks());
  HIP_TRY(ctx, hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double s = 0.0;
  for (double v : h) s += v;
  *out = s;
  return 0;
}

int do_bounds(chfsi_op* op, int steps, const double* v0_dev, const double* v0_host, uint64_t seed,
              double* b_upper, double* lmin) {
  chfsi_ctx* ctx = op->ctx;
  const HostTables& t = op->t;
  const int cf = t.cplx ? 2 : 1;
  const int prec = t.cplx ? CHFSI_C128 : CHFSI_F64;
  const int64_t nr = t.M * cf;  // reals per vector
  void* vb;
  CHECK(ws_get(ctx, WS_VEC, static_cast<size_t>(nr) * 3 * 8, &vb));
  double* v = static_cast<double*>(vb);
  double* vprev = v + nr;
  double* f = v + 2 * nr;
  if (v0_dev) {
    HIP_TRY(ctx, hipMemcpyAsync(v, v0_dev, nr * 8, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    std::vector<double> h(nr);
    if (v0_host) {
      std::memcpy(h.data(), v0_host, nr * 8);
    } else {
      SplitMix g{seed};
      for (auto& x : h) x = g.normal();
    }
    HIP_TRY(ctx, hipMemcpyAsync(v, h.data(), nr * 8, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  double nv;
  CHECK(dot_host(ctx, v, v, nr, &nv));
  if (!(nv > 0.0) || !std::isfinite(nv)) return fail(ctx, CHFSI_EINVAL, "Lanczos start vector is zero or non-finite");
  HIP_TRY(ctx, launch_axpby(0.0, v, 1.0 / std::sqrt(nv), v, nr, ctx->stream));
  std::vector<double> al, be;
  // f = H v ; alpha = v.f ; f -= alpha v
  HIP_TRY(ctx, launch_fill(f, t.M, cf, cf, prec, ctx->stream));
  CHECK(hx_step(op, prec, v, 1, nullptr, 1, f, 1, 1, 1.0, 0.0, 0.0, false));
  double alpha;
  CHECK(dot_host(ctx, v, f, nr, &alpha));
  HIP_TRY(ctx, launch_axpby(-alpha, v, 1.0, f, nr, ctx->stream));
  al.push_back(alpha);
  for (int k = 1; k < steps; ++k) {
    double bb;
    CHECK(dot_host(ctx, f, f, nr, &bb));
    const double beta = std::sqrt(bb);
    if (!(beta > 0.0)) break;
    // vprev <- v ; v <- f / beta ; f <- H v - beta vprev ; alpha ; f -= alpha v
    std::swap(v, vprev);
    HIP_TRY(ctx, launch_axpby(1.0 / beta, f, 0.0, v, nr, ctx->stream));
    HIP_TRY(ctx, launch_fill(f, t.M, cf, cf, prec, ctx->stream));
    CHECK(hx_step(op, prec, v, 1, nullptr, 1, f, 1, 1, 1.0, 0.0, 0.0, false));
    HIP_TRY(ctx, launch_axpby(-beta, vprev, 1.0, f, nr, ctx->stream));
    CHECK(dot_host(ctx, v, f, nr, &alpha));
    HIP_TRY(ctx, launch_axpby(-alpha, v, 1.0, f, nr, ctx->stream));
    al.push_back(alpha);
    be.push_back(beta);
  }
  double ff;
  CHECK(dot_host(ctx, f, f, nr, &ff));
  const int k = static_cast<int>(al.size());
  std::vector<double> T(static_cast<size_t>(k) * k, 0.0);
  for (int i = 0; i < k; ++i) T[i * k + i] = al[i];
  for (int i = 0; i + 1 < k; ++i) T[i * k + i + 1] = T[(i + 1) * k + i] = be[i];
  std::vector<double> ev = small_eigvals(T, k);
  if (b_upper) *b_upper = ev.back() + std::sqrt(ff);
  if (lmin) *lmin = ev.front();
  if (!std::isfinite(ev.back()) || !std::isfinite(ff)) return fail(ctx, CHFSI_EDIVERGE, "non-finite Lanczos run");
  return 0;
}

int check_block(chfsi_op* op, const void* X, int64_t ncols, int64_t ld) {
  if (!X) return fail(op->ctx, CHFSI_EINVAL, "null block pointer");
  if (ncols <= 0) return fail(op->ctx, CHFSI_EINVAL, "ncols must be positive");
  if (ld < ncols) return fail(op->ctx, CHFSI_EINVAL, "ld < ncols");
  if (ncols > op->t.M) return fail(op->ctx, CHFSI_EINVAL, "ncols > M");
  return 0;
}

double event_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return ms;
}


// ---- batched filter over many operators (one persistent launch per step) ----

struct BItem {
  chfsi_op* op;
  double* X;       // subspace block (double / complex double)
  int64_t ncols;   // logical columns
  int64_t ld;
  double a, b, aL;
};

std::string tune_key(int p, int prec, int64_t block) {
  return "gfx950:p" + std::to_string(p) + ":prec" + std::to_string(prec) + ":B" + std::to_string(block);
}

chfsi_ctx::Tuning tuning_for(chfsi_ctx* ctx, int p, int prec, int64_t block) {
  auto it = ctx->tuning.find(tune_key(p, prec, block));
  if (it != ctx->tuning.end()) return it->second;
  chfsi_ctx::Tuning t;
  t.grid_per_cu = 0;  // one workgroup per item: the hardware dispatcher balances the load
  (void)prec;
  return t;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int pinned_get(chfsi_ctx* ctx, size_t bytes, void** out) {
  if (ctx->pinned_size < bytes) {
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_size = 0;
    HIP_TRY(ctx, hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
    ctx->pinned_size = bytes;
  }
  *out = ctx->pinned;
  return 0;
}

void drop_graph(chfsi_ctx* ctx) {
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->gexec = nullptr;
  ctx->graph = nullptr;
  ctx->gkey.clear();
}

// Filters every item's block X (all columns, in rounds of `block` columns)
// with degree m on its own [a, b], aL.  Each Chebyshev step of a round is one
// persistent launch over all items (cell_hx_batched_kernel); the per-item
// recurrence scalars live in device descriptor tables written before the
// launch, so with use_graph the whole sequence is captured once into a
// hipGraph and replayed while the tables change.
int batched_filter(chfsi_ctx* ctx, const std::vector<BItem>& items, int m, int prec, int64_t block,
                   bool use_graph, const chfsi_ctx::Tuning* force = nullptr) {
  const int n = static_cast<int>(items.size());
  if (n == 0) return 0;
  const int p = items[0].op->t.p;
  const bool cplx = items[0].op->t.cplx;
  for (const BItem& it : items) {
    if (it.op->ctx != ctx) return fail(ctx, CHFSI_EINVAL, "operators of a batch must share the context");
    if (it.op->t.p != p || it.op->t.cplx != cplx)
      return fail(ctx, CHFSI_EINVAL, "operators of a batch must share order p and real/complex type");
    if (!prec_valid_for(it.op, prec)) return fail(ctx, CHFSI_EINVAL, "precision does not match the operators");
    if (prec == CHFSI_BF16) return fail(ctx, CHFSI_EINVAL, "batched filter supports F64, F32, C128, C64");
    if (!(it.aL < it.a && it.a < it.b)) return fail(ctx, CHFSI_EINVAL, "need aL < a < b for every item");
  }
  // deterministic assembly: each problem's filter on its own, colour class
  // by colour class (no batched launch, no graph)
  if (ctx->deterministic && !force) {
    for (const BItem& it : items) CHECK(do_filter(it.op, it.X, it.ncols, it.ld, m, it.a, it.b, it.aL, prec, block));
    return 0;
  }
  const int cf = cplx ? 2 : 1;
  const int sp = storage_of(prec);
  const int xprec = cplx ? CHFSI_C128 : CHFSI_F64;
  const size_t ebl = prec_bytes(sp);           // bytes per logical entry
  const size_t esc = is_single(prec) ? 4 : 8;  // bytes per real scalar
  std::vector<int64_t> Bq(n);
  int rounds = 0;
  for (int q = 0; q < n; ++q) {
    Bq[q] = (block <= 0 || block > items[q].ncols) ? items[q].ncols : block;
    rounds = std::max<int>(rounds, static_cast<int>((items[q].ncols + Bq[q] - 1) / Bq[q]));
  }
  // launch shape: tuned (or forced), else one workgroup per item and the
  // 32-column work item for blocks of at most 32 real columns
  const chfsi_ctx::Tuning tu = force ? *force : tuning_for(ctx, p, prec, block);
  int64_t widest = 0;
  for (int q = 0; q < n; ++q) widest = std::max(widest, Bq[q]);
  const int nt = (tu.col_tile == 32 || tu.col_tile == 64) ? tu.col_tile : (widest * cf <= 32 ? 32 : 64);
  // workspace: per item R0..R3, projector partials and coefficients
  std::vector<size_t> offR(n), offPart(n), offHP(n);
  std::vector<int64_t> ldhp(n);
  size_t total = 0;
  for (int q = 0; q < n; ++q) {
    const chfsi_op* op = items[q].op;
    offR[q] = total;
    total += align256(static_cast<size_t>(op->t.M) * Bq[q] * ebl) * 4;
    ldhp[q] = hp_ld(op, Bq[q]);
    offPart[q] = total;
    if (op->t.has_proj) total += align256(static_cast<size_t>(op->nchunks) * 4 * ldhp[q] * esc);
    offHP[q] = total;
    if (op->t.has_proj) total += align256(static_cast<size_t>(op->t.natoms) * 4 * ldhp[q] * esc);
  }
  const size_t db = hx_desc_bytes(prec);
  const size_t tab_desc = static_cast<size_t>(rounds) * m * n * db;
  const size_t tab_off = static_cast<size_t>(rounds) * (n + 1) * sizeof(int64_t);
  // the projections of all problems with projectors in two launches per step:
  // their descriptors per (round, step), chunk and row offsets per round
  const size_t tab_nl = static_cast<size_t>(rounds) * m * n * sizeof(NlLaunch);
  const size_t tab_nloff = static_cast<size_t>(rounds) * 2 * (n + 1) * sizeof(int64_t);
  const size_t nl_at = align256(tab_desc) + align256(tab_off);
  const size_t nloff_at = nl_at + align256(tab_nl);
  const size_t tab_bytes = nloff_at + tab_nloff;
  void *wsb, *tab, *host;
  CHECK(ws_get(ctx, WS_BATCH, total, &wsb));
  CHECK(ws_get(ctx, WS_BTAB, tab_bytes, &tab));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // the staging buffer is rewritten below
  CHECK(pinned_get(ctx, tab_bytes, &host));
  char* base = static_cast<char*>(wsb);
  auto R = [&](int q, int i) { return static_cast<void*>(base + offR[q] + align256(static_cast<size_t>(items[q].op->t.M) * Bq[q] * ebl) * i); };
  // host tables
  std::memset(host, 0, tab_bytes);
  char* hdesc = static_cast<char*>(host);
  int64_t* hoff = reinterpret_cast<int64_t*>(static_cast<char*>(host) + align256(tab_desc));
  NlLaunch* hnl = reinterpret_cast<NlLaunch*>(static_cast<char*>(host) + nl_at);
  int64_t* hnloff = reinterpret_cast<int64_t*>(static_cast<char*>(host) + nloff_at);
  std::vector<std::vector<int>> active(rounds);
  std::vector<std::vector<int64_t>> width(rounds);
  std::vector<int> nl_count(rounds, 0), nl_tiles(rounds, 0), nl_rowblk(rounds, 0);
  std::vector<int64_t> nl_chunks(rounds, 0), nl_rows(rounds, 0);
  for (int r = 0; r < rounds; ++r) {
    int64_t acc = 0;
    for (int q = 0; q < n; ++q) {
      const int64_t c0 = r * Bq[q];
      if (c0 >= items[q].ncols) continue;
      const int64_t nb = std::min<int64_t>(Bq[q], items[q].ncols - c0);
      active[r].push_back(q);
      width[r].push_back(nb);
    }
    const int na = static_cast<int>(active[r].size());
    for (int k = 0; k < na; ++k) {
      const int q = active[r][k];
      const chfsi_op* op = items[q].op;
      hoff[r * (n + 1) + k] = acc;
      acc += op->t.E * ((width[r][k] * cf + nt - 1) / nt);
      double c;
      std::vector<double> al, be;
      cheb_coeffs(m, items[q].a, items[q].b, items[q].aL, &c, al, be);
      const int64_t nb = width[r][k];
      for (int st = 1; st <= m; ++st) {
        HxLaunch L = make_hx(op, prec, R(q, (st - 1) % 4), nb, st >= 2 ? R(q, (st - 2) % 4) : nullptr, nb,
                             R(q, st % 4), nb, nb, al[st - 1], c, st >= 2 ? be[st - 1] : 0.0, st >= 2,
                             op->t.has_proj ? base + offHP[q] : nullptr, ldhp[q]);
        pack_hx_desc(L, prec, hdesc + ((static_cast<size_t>(r) * m + (st - 1)) * n + k) * db);
      }
      if (op->t.has_proj && op->nchunks > 0) {
        const int j = nl_count[r]++;
        hnloff[(static_cast<size_t>(r) * 2) * (n + 1) + j] = nl_chunks[r];
        hnloff[(static_cast<size_t>(r) * 2 + 1) * (n + 1) + j] = nl_rows[r];
        nl_chunks[r] += op->nchunks;
        nl_rows[r] += 4 * static_cast<int64_t>(op->t.natoms);
        nl_tiles[r] = std::max<int>(nl_tiles[r], static_cast<int>((nb + 63) / 64));   // logical columns
        nl_rowblk[r] = std::max<int>(nl_rowblk[r], static_cast<int>((ldhp[q] + 255) / 256));
        for (int st = 1; st <= m; ++st)
          hnl[(static_cast<size_t>(r) * m + (st - 1)) * n + j] =
              make_nl(op, R(q, (st - 1) % 4), nb, nb, base + offPart[q], base + offHP[q], ldhp[q]);
      }
    }
    for (int k = na; k <= n; ++k) hoff[r * (n + 1) + k] = acc;
    for (int j = nl_count[r]; j <= n; ++j) {
      hnloff[(static_cast<size_t>(r) * 2) * (n + 1) + j] = nl_chunks[r];
      hnloff[(static_cast<size_t>(r) * 2 + 1) * (n + 1) + j] = nl_rows[r];
    }
  }
  HIP_TRY(ctx, hipMemcpyAsync(tab, host, tab_bytes, hipMemcpyHostToDevice, ctx->stream));
  const char* dtab = static_cast<const char*>(tab);
  const int64_t* doff = reinterpret_cast<const int64_t*>(dtab + align256(tab_desc));

  // per-round algorithmic flops of the cell kernel (timed launches)
  std::vector<double> round_flops(rounds, 0.0);
  for (int r = 0; r < rounds; ++r)
    for (size_t k = 0; k < active[r].size(); ++k)
      round_flops[r] += cell_kernel_flops(items[active[r][k]].op, width[r][k]);
  // timed: HIP events around every batched cell-kernel launch (not inside a
  // captured graph), read by chfsi_kernel_time like the single-problem ones
  auto enqueue = [&](bool timed) -> int {
    for (int r = 0; r < rounds; ++r) {
      const int na = static_cast<int>(active[r].size());
      for (int k = 0; k < na; ++k) {
        const int q = active[r][k];
        const int64_t nb = width[r][k];
        const int64_t M = items[q].op->t.M;
        double* Xb = items[q].X + r * Bq[q] * cf;
        HIP_TRY(ctx, launch_convert(R(q, 0), nb * cf, sp, Xb, items[q].ld * cf, xprec, M, nb * cf, ctx->stream));
        for (int i = 1; i < 4; ++i) HIP_TRY(ctx, launch_fill(R(q, i), M, nb * cf, nb * cf, sp, ctx->stream));
      }
      for (int st = 1; st <= m; ++st) {
        if (nl_count[r] > 0) {
          NlBatch nb_;
          nb_.descs = dtab + nl_at + (static_cast<size_t>(r) * m + (st - 1)) * n * sizeof(NlLaunch);
          nb_.chunk_off = reinterpret_cast<const int64_t*>(dtab + nloff_at) + (static_cast<size_t>(r) * 2) * (n + 1);
          nb_.row_off = reinterpret_cast<const int64_t*>(dtab + nloff_at) + (static_cast<size_t>(r) * 2 + 1) * (n + 1);
          nb_.nprob = nl_count[r];
          nb_.total_chunks = nl_chunks[r];
          nb_.total_rows = nl_rows[r];
          nb_.max_col_tiles = nl_tiles[r];
          nb_.max_row_blocks = nl_rowblk[r];
          HIP_TRY(ctx, launch_nl_project_batched(nb_, prec, ctx->stream));
        }
        HxBatch hb;
        hb.p = p;
        hb.nt = nt;
        hb.descs = dtab + (static_cast<size_t>(r) * m + (st - 1)) * n * db;
        hb.item_off = doff + r * (n + 1);
        hb.nprob = na;
        // grid_per_cu > 0: a persistent grid of that many workgroups per CU;
        // 0: one workgroup per item of the round
        const int64_t nitems_r = hoff[r * (n + 1) + na];
        hb.grid = tu.grid_per_cu > 0 ? std::max(1, ctx->ncu * tu.grid_per_cu)
                                     : static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nitems_r, 0x7fffffff)));
        hb.contiguous = tu.contiguous;
        hb.one_per_item = tu.grid_per_cu == 0 && nitems_r <= 0x7fffffff;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timed) {
          HIP_TRY(ctx, hipEventCreate(&e0));
          HIP_TRY(ctx, hipEventCreate(&e1));
          HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
        }
        HIP_TRY(ctx, launch_cell_hx_batched(hb, prec, ctx->stream));
        if (timed) {
          HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
          ctx->pending.emplace_back(e0, e1);
          ctx->pending_flops.push_back(round_flops[r]);
        }
      }
      for (int k = 0; k < na; ++k) {
        const int q = active[r][k];
        const int64_t nb = width[r][k];
        double* Xb = items[q].X + r * Bq[q] * cf;
        HIP_TRY(ctx, launch_convert(Xb, items[q].ld * cf, xprec, R(q, m % 4), nb * cf, sp, items[q].op->t.M,
                                    nb * cf, ctx->stream));
      }
    }
    return 0;
  };
  if (!use_graph) return enqueue(ctx->timing);
  // the graph is keyed by everything its nodes point at
  std::ostringstream key;
  key << m << ":" << prec << ":" << block << ":" << wsb << ":" << tab << ":" << tu.grid_per_cu << ":" << tu.contiguous
      << ":" << nt;
  // operators by id (never reused within the context), so that an operator
  // built at a destroyed one's address cannot match a stale graph
  for (const BItem& it : items) key << ":op" << it.op->id << "," << it.X << "," << it.ncols << "," << it.ld;
  if (key.str() != ctx->gkey || !ctx->gexec) {
    drop_graph(ctx);
    // Capture on the context's private stream (the caller's stream may be the
    // legacy default stream, which cannot be captured); capturing records the
    // sequence without running it, and the graph is launched on ctx->stream.
    if (!ctx->cap_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipStream_t user = ctx->stream;
    HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
    ctx->stream = ctx->cap_stream;
    const int rc = enqueue(false);
    ctx->stream = user;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (rc < 0) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(ctx, CHFSI_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
    ctx->graph = g;
    HIP_TRY(ctx, hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
    ctx->gkey = key.str();
  }
  HIP_TRY(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
  return 0;
}

int load_tuning_file(chfsi_ctx* ctx, const std::string& path) {
  std::ifstream f(path);
  if (!f) return 0;
  std::string line;
  while (std::getline(f, line)) {
    const size_t k0 = line.find("\"key\": \"");
    if (k0 == std::string::npos) continue;
    const size_t k1 = line.find('"', k0 + 8);
    chfsi_ctx::Tuning t;
    const size_t g = line.find("\"grid_per_cu\": ");
    const size_t c = line.find("\"contiguous\": ");
    const size_t ms = line.find("\"ms\": ");
    const size_t ct = line.find("\"col_tile\": ");
    if (k1 == std::string::npos || g == std::string::npos || c == std::string::npos) continue;
    t.grid_per_cu = std::atoi(line.c_str() + g + 15);
    t.contiguous = std::atoi(line.c_str() + c + 14);
    if (ms != std::string::npos) t.ms = std::atof(line.c_str() + ms + 6);
    if (ct != std::string::npos) t.col_tile = std::atoi(line.c_str() + ct + 12);   // absent: the default rule
    if (t.col_tile != 0 && t.col_tile != 32 && t.col_tile != 64) continue;
    if (t.grid_per_cu >= 0 && t.grid_per_cu <= 16) ctx->tuning[line.substr(k0 + 8, k1 - k0 - 8)] = t;
  }
  return 0;
}

int save_tuning_file(chfsi_ctx* ctx, const std::string& path) {
  std::ofstream f(path);
  if (!f) return fail(ctx, CHFSI_EINVAL, "cannot write tuning cache " + path);
  f << "[\n";
  size_t i = 0;
  for (const auto& kv : ctx->tuning) {
    f << "{\"key\": \"" << kv.first << "\", \"grid_per_cu\": " << kv.second.grid_per_cu
      << ", \"contiguous\": " << kv.second.contiguous << ", \"col_tile\": " << kv.second.col_tile
      << ", \"ms\": " << kv.second.ms << "}"
      << (++i < ctx->tuning.size() ? "," : "") << "\n";
  }
  f << "]\n";
  return 0;
}

}  // namespace

namespace {

// Mixed-precision schedule: the next filter precision after a pass whose
// residual history is r[0..k] (k >= 1), or prec itself.
int next_prec(int prec, const double* r, int k, double b) {
  int up = prec;
  double u = 0.0;
  if (prec == CHFSI_BF16) { up = CHFSI_F32; u = std::ldexp(1.0, -8); }
  else if (prec == CHFSI_F32) { up = CHFSI_F64; u = std::ldexp(1.0, -24); }
  else if (prec == CHFSI_C64) { up = CHFSI_C128; u = std::ldexp(1.0, -24); }
  else return prec;
  const bool floor_reached = r[k] <= 4.0 * u * b;
  const bool growing = k >= 2 && r[k] > r[k - 1] && r[k - 1] > r[k - 2];
  return (floor_reached || growing) ? up : prec;
}

// ---- SCF loop helpers --------------------------------------------------------

// Device tables of the SCF loop, built once per operator: the build-time
// nodal potential V_ext, M^1/2, M, the diagonal of D K D (the Jacobi
// preconditioner of the Hartree problem) and a zero vector.
int scf_tables(chfsi_op* op) {
  if (op->scf_tab) return 0;
  chfsi_ctx* ctx = op->ctx;
  const HostTables& t = op->t;
  const int64_t M = t.M;
  const int p = t.p, q = p + 1, n = t.n;
  std::vector<double> h(static_cast<size_t>(5) * M, 0.0);
  double* vext = h.data();
  double* sqm = vext + M;
  double* mm = sqm + M;
  double* kd = mm + M;
  // the build-time potential without the |k|^2 / 2 of a Bloch operator
  // (chfsi_op_set_potential adds it back)
  const double k2 = 0.5 * (t.k[0] * t.k[0] + t.k[1] * t.k[1] + t.k[2] * t.k[2]);
  for (int64_t j = 0; j < M; ++j) {
    vext[j] = t.vdiag[j] - k2;
    sqm[j] = 1.0 / t.dscale[j];
    mm[j] = sqm[j] * sqm[j];
  }
  // diag(D K D)_j = sum over the (cell, local index) pairs of node j of
  // 2 A_ll, A = D_c (K^c / 2) D_c; along each axis a vertex-type index
  // (i mod p = 0) is local index 0 of one cell and p of its neighbour
  auto opts = [&](int i, int* o) -> int {
    if (i % p == 0) {
      o[0] = 0;
      o[1] = p;
      return 2;
    }
    o[0] = i % p;
    return 1;
  };
  for (int iz = 0; iz < n; ++iz)
    for (int iy = 0; iy < n; ++iy)
      for (int ix = 0; ix < n; ++ix) {
        int ox[2], oy[2], oz[2];
        const int nx = opts(ix, ox), ny = opts(iy, oy), nz = opts(iz, oz);
        double s = 0.0;
        for (int c = 0; c < nz; ++c)
          for (int b = 0; b < ny; ++b)
            for (int a = 0; a < nx; ++a) {
              const int64_t l = ox[a] + q * (oy[b] + static_cast<int64_t>(q) * oz[c]);
              s += 2.0 * t.cell_re[l * t.mcell + l];
            }
        kd[ix + static_cast<int64_t>(n) * (iy + static_cast<int64_t>(n) * iz)] = s;
      }
  double* d;
  CHECK(upload(op, h, &d));
  op->scf_tab = d;
  return 0;
}

// q = (D K D) u on the operator's mesh, one vector: the cell stiffness by sum
// factorisation of its 1D factors (a 64-column MFMA tile would waste 63/64
// of its work on a single column).
int apply_stiffness(chfsi_op* op, const double* u, double* qv) {
  chfsi_ctx* ctx = op->ctx;
  const HostTables& t = op->t;
  HIP_TRY(ctx, launch_fill(qv, t.M, 1, 1, CHFSI_F64, ctx->stream));
  if (!ctx->deterministic) {
    HIP_TRY(ctx, launch_stiffness(u, op->dscale, qv, t.p, t.ncell, t.K1d.data(), t.M1d.data(), ctx->stream));
    return 0;
  }
  // deterministic assembly: colour class by colour class, as for H~X
  CHECK(build_colours(op));
  for (size_t k = 0; k + 1 < op->colour_off.size(); ++k)
    HIP_TRY(ctx, launch_stiffness(u, op->dscale, qv, t.p, t.ncell, t.K1d.data(), t.M1d.data(), ctx->stream,
                                  op->colour_cells + op->colour_off[k], op->colour_off[k + 1] - op->colour_off[k]));
  return 0;
}

// Hartree potential: D K D u = 4 pi M^1/2 (rho - rho_bar), v_H = D u, by
// Jacobi-preconditioned CG with the null vector M^1/2 1 projected out.
// w: 6 M scratch values.
// warm: start from the potential already in vh (the previous SCF step's)
// instead of zero; the stopping rule stays relative to the right-hand side.
int hartree_solve(chfsi_op* op, const double* rho, double* vh, double tol, int maxit, double* w, int* iters,
                  double* relres, bool warm = false) {
  chfsi_ctx* ctx = op->ctx;
  const int64_t M = op->t.M;
  hipStream_t st = ctx->stream;
  CHECK(scf_tables(op));
  const double* sqm = op->scf_tab + M;
  const double* mm = op->scf_tab + 2 * M;
  const double* kd = op->scf_tab + 3 * M;
  double *u = w, *r = w + M, *z = w + 2 * M, *pv = w + 3 * M, *qv = w + 4 * M, *b = w + 5 * M;
  double q_tot = 0.0, m_tot = 0.0, zz = 0.0;
  CHECK(dot_host(ctx, mm, rho, M, &q_tot));
  CHECK(dot_host(ctx, sqm, sqm, M, &zz));   // = sum M
  m_tot = zz;
  HIP_TRY(ctx, launch_hartree_rhs(rho, q_tot / m_tot, sqm, b, M, st));
  auto project = [&](double* x) -> int {   // x -= (x . n) n, n = M^1/2 1 / |.|
    double xn = 0.0;
    CHECK(dot_host(ctx, x, sqm, M, &xn));
    HIP_TRY(ctx, launch_axpby(-xn / zz, sqm, 1.0, x, M, st));
    return 0;
  };
  CHECK(project(b));
  double bb = 0.0;
  CHECK(dot_host(ctx, b, b, M, &bb));
  HIP_TRY(ctx, launch_convert(r, 1, CHFSI_F64, b, 1, CHFSI_F64, M, 1, st));
  double rr = bb;
  if (warm) {
    // u = M^1/2 v (v = D u), kept orthogonal to the constant mode; r = b - A u
    HIP_TRY(ctx, launch_emul(vh, sqm, u, M, st));
    CHECK(project(u));
    CHECK(apply_stiffness(op, u, qv));
    HIP_TRY(ctx, launch_axpby(-1.0, qv, 1.0, r, M, st));
    CHECK(project(r));
    CHECK(dot_host(ctx, r, r, M, &rr));
  } else {
    HIP_TRY(ctx, launch_fill(u, M, 1, 1, CHFSI_F64, st));
  }
  HIP_TRY(ctx, launch_ediv(r, kd, z, M, st));
  CHECK(project(z));
  HIP_TRY(ctx, launch_convert(pv, 1, CHFSI_F64, z, 1, CHFSI_F64, M, 1, st));
  double rz = 0.0;
  CHECK(dot_host(ctx, r, z, M, &rz));
  // the iterations keep their scalars on the device (launch_cg_iteration);
  // the host reads the residual history once per kCheck iterations, so a
  // solve runs up to kCheck - 1 iterations past the stopping point
  constexpr int kCheck = 8;
  // scalars, residual history, and (deterministic mode) the dot products'
  // block partials, 5 x 256 values
  void* scv;
  CHECK(ws_get(ctx, WS_CG, (8 + kCheck + 5 * 256) * 8, &scv));
  double* sc = static_cast<double*>(scv);
  double* hist = sc + 8;
  double* part = ctx->deterministic ? sc + 8 + kCheck : nullptr;
  const double sc0[8] = {rz, 0.0, 0.0, 0.0, 0.0, zz, 0.0, 0.0};
  HIP_TRY(ctx, hipMemcpyAsync(sc, sc0, sizeof(sc0), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  int it = 0;
  const double stop = tol * tol * bb;
  double hh[kCheck];
  while (it < maxit && rr > stop && bb > 0.0) {
    const int k = std::min(kCheck, maxit - it);
    for (int j = 0; j < k; ++j) {
      CHECK(apply_stiffness(op, pv, qv));
      HIP_TRY(ctx, launch_cg_iteration(u, r, z, pv, qv, kd, sqm, sc, hist, j, M, st, part));
    }
    HIP_TRY(ctx, hipMemcpyAsync(hh, hist, k * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    it += k;
    rr = hh[k - 1];
    if (!(rr == rr)) return fail(ctx, CHFSI_EDIVERGE, "Hartree CG produced NaN");
  }
  HIP_TRY(ctx, launch_ediv(u, sqm, vh, M, st));   // v = D u
  if (iters) *iters = it;
  if (relres) *relres = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
  return 0;
}

// Checks the Ritz values of a pass: they must be finite and, since every Ritz
// value lies in [lambda_min, lambda_max] (Cauchy interlacing), none may lie
// above a valid upper bound b of the spectrum.  A Ritz value above b shows
// that b is below lambda_max: the filter then amplifies the unwanted top of
// the spectrum instead of damping it (Section 3.1), and the iteration
// diverges.
int check_ritz(chfsi_ctx* ctx, const double* th, const double* r, int64_t N, double b) {
  for (int64_t i = 0; i < N; ++i)
    if (!std::isfinite(th[i]) || (r && !std::isfinite(r[i])))
      return fail(ctx, CHFSI_EDIVERGE, "non-finite Ritz values or residuals");
  for (int64_t i = 0; i < N; ++i)
    if (b > 0.0 && th[i] > b + 1e-9 * std::fabs(b))
      return fail(ctx, CHFSI_EDIVERGE, "a Ritz value lies above the upper bound b: b is below lambda_max");
  return 0;
}

void record_hist(const chfsi_params& p, int i, double t_ms, double maxr, int prec, const double* th, int64_t N) {
  if (i < 0 || i >= p.hist_len) return;
  if (p.hist_time_ms) p.hist_time_ms[i] = t_ms;
  if (p.hist_max_resid) p.hist_max_resid[i] = maxr;
  if (p.hist_prec) p.hist_prec[i] = prec;
  if (p.hist_theta) std::memcpy(p.hist_theta + static_cast<int64_t>(i) * N, th, N * 8);
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* chfsi_version(void) { return "chfsi 0.1 (gfx950)"; }

int32_t chfsi_next_prec(int32_t prec, const double* max_resid, int32_t k, double b_upper) {
  if (!max_resid || k < 1) return prec;
  return next_prec(prec, max_resid, k, b_upper);
}

int chfsi_abi_sizes(int64_t* system, int64_t* params, int64_t* stats) {
  if (system) *system = static_cast<int64_t>(sizeof(chfsi_system));
  if (params) *params = static_cast<int64_t>(sizeof(chfsi_params));
  if (stats) *stats = static_cast<int64_t>(sizeof(chfsi_stats));
  return CHFSI_OK;
}

int chfsi_ctx_create(chfsi_ctx** out, int device, void* hip_stream) {
  if (!out) return fail(nullptr, CHFSI_EINVAL, "null output pointer");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return fail(nullptr, CHFSI_EHIP, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(nullptr, CHFSI_EINVAL, "device index out of range");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, CHFSI_EHIP, "hipSetDevice failed");
  std::unique_ptr<chfsi_ctx> c(new chfsi_ctx());
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(nullptr, CHFSI_EHIP, "hipGetDeviceProperties failed");
  c->ncu = prop.multiProcessorCount;
  // the fixed scratch of chfsi_apply_noalloc(): its address on this device
  // (device current), kept for the context's lifetime
  {
    const hipError_t e = scratch_address(&c->scratch);
    if (e != hipSuccess) {
      c->scratch = nullptr;
      c->scratch_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    }
  }
  if (rocblas_create_handle(&c->blas) != rocblas_status_success)
    return fail(nullptr, CHFSI_EHIP, "rocblas_create_handle failed");
  if (rocblas_set_stream(c->blas, c->stream) != rocblas_status_success)
    return fail(nullptr, CHFSI_EHIP, "rocblas_set_stream failed");
  *out = c.release();
  return 0;
}

int chfsi_ctx_destroy(chfsi_ctx* ctx) {
  if (!ctx) return 0;
  if (!ctx->live_ops.empty() || !ctx->live_mlps.empty())
    return fail(ctx, CHFSI_EINVAL,
                std::to_string(ctx->live_ops.size()) + " operator(s) and " + std::to_string(ctx->live_mlps.size()) +
                    " network(s) of this context are still alive: destroy them first");
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& pr : ctx->pending) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  for (int i = 0; i < WS_COUNT; ++i)
    if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
  if (ctx->blas) rocblas_destroy_handle(ctx->blas);
  delete ctx;
  return 0;
}

const char* chfsi_last_error(const chfsi_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int chfsi_sync(chfsi_ctx* ctx) {
  if (!ctx) return CHFSI_EINVAL;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return 0;
}

int chfsi_op_build(chfsi_ctx* ctx, const chfsi_system* sys, chfsi_op** out) {
  if (!ctx) return CHFSI_EINVAL;
  if (!sys || !out) return fail(ctx, CHFSI_EINVAL, "null argument");
  *out = nullptr;
  if (sys->p < kMinOrder || sys->p > kMaxOrder) return fail(ctx, CHFSI_EINVAL, "order p must be in [2, 7]");
  if (sys->natoms > 0 && (!sys->pos || !sys->Z || !sys->s)) return fail(ctx, CHFSI_EINVAL, "null atom arrays");
  if (sys->has_proj && sys->natoms > 0 && (!sys->w || !sys->h_s || !sys->h_p))
    return fail(ctx, CHFSI_EINVAL, "null projector arrays");
  // every floating-point input must be finite: a NaN or an infinity would
  // reach every table built from it
  {
    bool fin = std::isfinite(sys->L) && std::isfinite(sys->k[0]) && std::isfinite(sys->k[1]) &&
               std::isfinite(sys->k[2]);
    for (int i = 0; i < sys->natoms && fin; ++i) {
      fin = std::isfinite(sys->pos[3 * i]) && std::isfinite(sys->pos[3 * i + 1]) &&
            std::isfinite(sys->pos[3 * i + 2]) && std::isfinite(sys->Z[i]) && std::isfinite(sys->s[i]);
      if (fin && sys->has_proj)
        fin = std::isfinite(sys->w[i]) && std::isfinite(sys->h_s[i]) && std::isfinite(sys->h_p[i]);
    }
    if (!fin) return fail(ctx, CHFSI_EINVAL, "non-finite value (NaN or infinity) in the system description");
  }
  if (sys->ncell < 1 || !(sys->L > 0.0) || sys->natoms < 0) return fail(ctx, CHFSI_EINVAL, "bad mesh size");
  const int64_t n = static_cast<int64_t>(sys->ncell) * sys->p;
  if (n * n * n >= (1LL << 29)) return fail(ctx, CHFSI_EINVAL, "mesh too large (node ids must stay below 2^29)");
  for (int i = 0; i < sys->natoms; ++i) {
    if (!(sys->s[i] > 0.0)) return fail(ctx, CHFSI_EINVAL, "Gaussian widths must be positive");
    if (sys->has_proj && !(sys->w[i] > 0.0)) return fail(ctx, CHFSI_EINVAL, "projector widths must be positive");
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  std::unique_ptr<chfsi_op> op(new chfsi_op());
  op->ctx = ctx;
  HostTables& t = op->t;
  std::string e = build_tables(*sys, t);
  if (!e.empty()) return fail(ctx, CHFSI_EINVAL, e);
  auto cleanup = [&]() {
    for (void* p : op->allocs) (void)hipFree(p);
    op->allocs.clear();
  };
  int rc = 0;
  do {
    std::vector<double> sw(static_cast<size_t>(t.mpad / 16) * (t.mpad / 4) * 64);
    swizzle_cell_matrix(t.cell_re.data(), t.mcell, t.mpad, sw.data());
    double* d;
    if ((rc = upload(op.get(), sw, &d)) < 0) break;
    op->A64 = d;
    if ((rc = upload_f32(op.get(), sw, &op->A32)) < 0) break;
    if (!t.cplx) {
      const int mp32 = mpad32_of(t.p);
      std::vector<uint16_t> bf(static_cast<size_t>(mp32 / 16) * (mp32 / 32) * 64 * 8);
      swizzle_cell_matrix_bf16(t.cell_re.data(), t.mcell, bf.data());
      uint16_t* db;
      if ((rc = upload(op.get(), bf, &db)) < 0) break;
      op->Abf = db;
    }
    if (t.cplx) {
      swizzle_cell_matrix(t.cell_im.data(), t.mcell, t.mpad, sw.data());
      if ((rc = upload(op.get(), sw, &d)) < 0) break;
      op->Ai64 = d;
      if ((rc = upload_f32(op.get(), sw, &op->Ai32)) < 0) break;
    }
    if ((rc = upload(op.get(), t.vdiag, &op->vdiag)) < 0) break;
    if ((rc = upload(op.get(), t.dscale, &op->dscale)) < 0) break;
    if (t.has_proj) {
      if ((rc = upload(op.get(), t.atom_ptr, &op->atom_ptr)) < 0) break;
      if ((rc = upload(op.get(), t.atom_node, &op->atom_node)) < 0) break;
      if ((rc = upload(op.get(), t.atom_val, &op->atom_val)) < 0) break;
      if ((rc = upload(op.get(), t.hcoef, &op->hcoef)) < 0) break;
      // fixed-size chunks of each atom's node list
      std::vector<int32_t> ca, acp(1, 0);
      std::vector<int64_t> cb;
      for (int a = 0; a < t.natoms; ++a) {
        for (int64_t b = t.atom_ptr[a]; b < t.atom_ptr[a + 1]; b += 512) {
          ca.push_back(a);
          cb.push_back(b);
        }
        acp.push_back(static_cast<int32_t>(ca.size()));
      }
      op->nchunks = static_cast<int>(ca.size());
      if ((rc = upload(op.get(), ca, &op->chunk_atom)) < 0) break;
      if ((rc = upload(op.get(), cb, &op->chunk_begin)) < 0) break;
      if ((rc = upload(op.get(), acp, &op->atom_chunk_ptr)) < 0) break;
      if ((rc = upload(op.get(), t.pair_ptr, &op->pair_ptr)) < 0) break;
      if ((rc = upload(op.get(), t.pair_atom, &op->pair_atom)) < 0) break;
      op->npairs = static_cast<int64_t>(t.pair_atom.size());
      if ((rc = upload(op.get(), t.pair_re, &d)) < 0) break;
      op->pair_re64 = d;
      if ((rc = upload_f32(op.get(), t.pair_re, &op->pair_re32)) < 0) break;
      if (t.cplx) {
        if ((rc = upload(op.get(), t.pair_im, &d)) < 0) break;
        op->pair_im64 = d;
        if ((rc = upload_f32(op.get(), t.pair_im, &op->pair_im32)) < 0) break;
      }
    }
  } while (0);
  if (rc < 0) {
    cleanup();
    return rc;
  }
  // large projector arrays live on the device only
  std::vector<double>().swap(t.atom_val);
  std::vector<int32_t>().swap(t.atom_node);
  std::vector<double>().swap(t.pair_re);
  std::vector<double>().swap(t.pair_im);
  // deterministic assembly already on: the colour classes now, so that no
  // later call has to allocate them (operators with one cell per side have
  // none and are refused at their first H~.X)
  if (ctx->deterministic && t.ncell >= 2) {
    if ((rc = build_colours(op.get())) < 0) {
      cleanup();
      return rc;
    }
  }
  op->id = ctx->next_op_id++;
  ctx->live_ops.insert(op.get());
  *out = op.release();
  return 0;
}

// Replaces the nodal (collocated) local potential of a freshly built
// operator by the per-cell Gauss-quadrature one (Section 4.2): V~ on the
// device, K^loc = P V~ as one GEMM, per-cell matrices A_e = A + D_c K^loc_e D_c
// in FP64 and FP32, and a diagonal that keeps only |k|^2 / 2.
int build_quadrature_potential(chfsi_op* op, const chfsi_system* sys) {
  chfsi_ctx* ctx = op->ctx;
  HostTables& t = op->t;
  const int p = t.p, q = p + 1, nq = q * q * q, mc = t.mcell, mp = t.mpad;
  const int64_t E = t.E, msym = static_cast<int64_t>(mc) * (mc + 1) / 2;
  if (msym * E >= (int64_t{1} << 31) || static_cast<int64_t>(nq) * E >= (int64_t{1} << 31))
    return fail(ctx, CHFSI_EINVAL, "mesh too large for the per-cell potential GEMM (32-bit dimensions)");
  // basis products at the Gauss points, pairs j <= k (j-major) by points
  std::vector<double> Nq(static_cast<size_t>(nq) * mc);
  for (int qp = 0; qp < nq; ++qp) {
    const int qx = qp % q, qy = (qp / q) % q, qz = qp / (q * q);
    for (int l = 0; l < mc; ++l) {
      const int ax = l % q, ay = (l / q) % q, az = l / (q * q);
      Nq[static_cast<size_t>(qp) * mc + l] = t.interp[qx * q + ax] * t.interp[qy * q + ay] * t.interp[qz * q + az];
    }
  }
  std::vector<double> P(static_cast<size_t>(msym) * nq);
  for (int qp = 0; qp < nq; ++qp) {
    const double* n = &Nq[static_cast<size_t>(qp) * mc];
    int64_t r = 0;
    for (int j = 0; j < mc; ++j)
      for (int k = j; k < mc; ++k) P[static_cast<size_t>(qp) * msym + r++] = n[j] * n[k];
  }
  // Gauss rule and the cell's Loewdin scale per local node
  std::vector<double> gq(q), gw(q), Dl(mc);
  gauss_legendre_rule(q, gq, gw);
  for (int l = 0; l < mc; ++l) {
    const int ax = l % q, ay = (l / q) % q, az = l / (q * q);
    const int64_t nd = (ax % t.n) + static_cast<int64_t>(t.n) * ((ay % t.n) + static_cast<int64_t>(t.n) * (az % t.n));
    Dl[l] = t.dscale[nd];
  }
  std::vector<double> atoms(static_cast<size_t>(std::max(1, sys->natoms)) * 8, 0.0);
  for (int a = 0; a < sys->natoms; ++a) {
    atoms[8 * a + 0] = sys->pos[3 * a];
    atoms[8 * a + 1] = sys->pos[3 * a + 1];
    atoms[8 * a + 2] = sys->pos[3 * a + 2];
    atoms[8 * a + 3] = sys->Z[a];
    atoms[8 * a + 4] = sys->s[a];
  }
  std::vector<void*> tmp;
  auto dalloc = [&](size_t bytes, void** out) -> int {
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) return fail(ctx, CHFSI_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    tmp.push_back(*out);
    return 0;
  };
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(ctx->stream);
    for (void* v : tmp) (void)hipFree(v);
  };
  int rc = 0;
  do {
    void *dP, *dV, *dK, *dA, *dgq, *dgw, *dD, *dAt;
    if ((rc = dalloc(P.size() * 8, &dP)) < 0) break;
    if ((rc = dalloc(static_cast<size_t>(nq) * E * 8, &dV)) < 0) break;
    if ((rc = dalloc(static_cast<size_t>(msym) * E * 8, &dK)) < 0) break;
    if ((rc = dalloc(q * 8, &dgq)) < 0 || (rc = dalloc(q * 8, &dgw)) < 0) break;
    if ((rc = dalloc(mc * 8, &dD)) < 0 || (rc = dalloc(atoms.size() * 8, &dAt)) < 0) break;
    hipStream_t st = ctx->stream;
    if (hipMemcpy(dP, P.data(), P.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dgq, gq.data(), q * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dgw, gw.data(), q * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dD, Dl.data(), mc * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dAt, atoms.data(), atoms.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(ctx, CHFSI_EHIP, "upload of the quadrature tables failed");
      break;
    }
    if (launch_gauss_potential(static_cast<double*>(dAt), sys->natoms, t.L, t.ncell, p, static_cast<double*>(dgq),
                               static_cast<double*>(dgw), static_cast<double*>(dV), st) != hipSuccess) {
      rc = fail(ctx, CHFSI_EHIP, "Gauss-point potential launch failed");
      break;
    }
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(ctx->blas, rocblas_operation_none, rocblas_operation_none, static_cast<rocblas_int>(msym),
                      static_cast<rocblas_int>(E), nq, &one, static_cast<double*>(dP),
                      static_cast<rocblas_int>(msym), static_cast<double*>(dV), nq, &zero, static_cast<double*>(dK),
                      static_cast<rocblas_int>(msym)) != rocblas_status_success) {
      rc = fail(ctx, CHFSI_EHIP, "cell potential GEMM failed");
      break;
    }
    const int64_t per = static_cast<int64_t>(mp) * mp;
    hipError_t e = hipMalloc(&dA, static_cast<size_t>(E) * per * 8);
    if (e != hipSuccess) {
      rc = fail(ctx, CHFSI_ENOMEM, "per-cell matrices do not fit");
      break;
    }
    op->allocs.push_back(dA);
    if (launch_assemble_cell_matrices(static_cast<const double*>(op->A64), static_cast<double*>(dK), msym,
                                      static_cast<double*>(dD), mc, mp, E, static_cast<double*>(dA), st) != hipSuccess) {
      rc = fail(ctx, CHFSI_EHIP, "cell matrix assembly launch failed");
      break;
    }
    void* dA32;
    e = hipMalloc(&dA32, static_cast<size_t>(E) * per * 4);
    if (e != hipSuccess) {
      rc = fail(ctx, CHFSI_ENOMEM, "per-cell FP32 matrices do not fit");
      break;
    }
    op->allocs.push_back(dA32);
    if (launch_convert(dA32, per, CHFSI_F32, dA, per, CHFSI_F64, E, per, st) != hipSuccess) {
      rc = fail(ctx, CHFSI_EHIP, "cell matrix conversion launch failed");
      break;
    }
    // the diagonal keeps |k|^2 / 2 only
    const double k2 = 0.5 * (t.k[0] * t.k[0] + t.k[1] * t.k[1] + t.k[2] * t.k[2]);
    t.vdiag.assign(static_cast<size_t>(t.M), k2);
    if (hipMemcpy(op->vdiag, t.vdiag.data(), t.M * 8, hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(ctx, CHFSI_EHIP, "diagonal upload failed");
      break;
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(ctx, CHFSI_EHIP, "quadrature potential build failed");
      break;
    }
    op->A64 = dA;
    op->A32 = dA32;
    op->astride = per;
  } while (0);
  cleanup();
  return rc;
}

int chfsi_op_build_quadrature(chfsi_ctx* ctx, const chfsi_system* sys, chfsi_op** out) {
  if (!ctx) return CHFSI_EINVAL;
  if (!sys || !out) return fail(ctx, CHFSI_EINVAL, "null argument");
  CHECK(chfsi_op_build(ctx, sys, out));
  const int rc = build_quadrature_potential(*out, sys);
  if (rc < 0) {
    chfsi_op_destroy(*out);
    *out = nullptr;
  }
  return rc;
}

int chfsi_op_destroy(chfsi_op* op) {
  if (!op) return 0;
  chfsi_ctx* ctx = op->ctx;
  (void)hipStreamSynchronize(ctx->stream);
  // a captured batched graph may point at this operator's tables
  if (ctx->gkey.find(":op" + std::to_string(op->id) + ",") != std::string::npos) drop_graph(ctx);
  ctx->live_ops.erase(op);
  for (void* p : op->allocs) (void)hipFree(p);
  delete op;
  return 0;
}

int chfsi_op_info(const chfsi_op* op, int64_t* M, int64_t* E, int32_t* mcell, int32_t* nproj, int64_t* npairs,
                  int32_t* is_complex) {
  if (!op) return CHFSI_EINVAL;
  if (M) *M = op->t.M;
  if (E) *E = op->t.E;
  if (mcell) *mcell = op->t.mcell;
  if (nproj) *nproj = op->t.has_proj ? 4 * op->t.natoms : 0;
  if (npairs) *npairs = op->npairs;
  if (is_complex) *is_complex = op->t.cplx ? 1 : 0;
  return 0;
}

int chfsi_op_tables(const chfsi_op* op, double* xyz, double* cell_re, double* cell_im, double* vdiag,
                    double* dscale) {
  if (!op) return CHFSI_EINVAL;
  const HostTables& t = op->t;
  if (xyz) {
    const int64_t n = t.n;
    for (int64_t j = 0; j < t.M; ++j) {
      xyz[3 * j] = t.x1d[j % n];
      xyz[3 * j + 1] = t.x1d[(j / n) % n];
      xyz[3 * j + 2] = t.x1d[j / (n * n)];
    }
  }
  if (cell_re) std::memcpy(cell_re, t.cell_re.data(), t.cell_re.size() * 8);
  if (cell_im) {
    if (t.cplx) std::memcpy(cell_im, t.cell_im.data(), t.cell_im.size() * 8);
    else std::memset(cell_im, 0, static_cast<size_t>(t.mcell) * t.mcell * 8);
  }
  if (vdiag) std::memcpy(vdiag, t.vdiag.data(), t.M * 8);
  if (dscale) std::memcpy(dscale, t.dscale.data(), t.M * 8);
  return 0;
}

int chfsi_apply(chfsi_op* op, const void* X, void* Y, int64_t ncols, int64_t ld, int32_t prec) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  CHECK(check_block(op, X, ncols, ld));
  if (!Y) return fail(ctx, CHFSI_EINVAL, "null output");
  if (!prec_valid_for(op, prec)) return fail(ctx, CHFSI_EINVAL, "precision does not match the operator");
  if (X == Y) return fail(ctx, CHFSI_EINVAL, "X and Y must not overlap");
  const int cf = op->t.cplx ? 2 : 1;
  const int sp = storage_of(prec);
  HIP_TRY(ctx, launch_fill(Y, op->t.M, ncols * cf, ld * cf, sp, ctx->stream));
  return hx_step(op, prec, X, ld, nullptr, ld, Y, ld, ncols, 1.0, 0.0, 0.0, false);
}

int chfsi_apply_noalloc(chfsi_op* op, const void* X, void* Y, int64_t ncols, int64_t ld, int32_t prec) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  CHECK(check_block(op, X, ncols, ld));
  if (!Y) return fail(ctx, CHFSI_EINVAL, "null output");
  if (!prec_valid_for(op, prec)) return fail(ctx, CHFSI_EINVAL, "precision does not match the operator");
  if (X == Y) return fail(ctx, CHFSI_EINVAL, "X and Y must not overlap");
  const HostTables& t = op->t;
  const int cf = t.cplx ? 2 : 1;
  const int sp = storage_of(prec);
  // scratch layout: chunk partials (nchunks*4 x ldhp), then h P (natoms*4 x ldhp)
  const size_t eb = is_single(prec) ? 4 : 8;
  const int64_t ldhp = t.has_proj ? hp_ld(op, ncols) : 0;
  const size_t part_bytes = t.has_proj ? align256(static_cast<size_t>(op->nchunks) * 4 * ldhp * eb) : 0;
  const size_t need = t.has_proj ? part_bytes + static_cast<size_t>(t.natoms) * 4 * ldhp * eb : 0;
  if (need > kScratchBytes)
    return fail(ctx, CHFSI_EINVAL,
                "chfsi_apply_noalloc needs " + std::to_string(need) + " bytes of scratch for " +
                    std::to_string(ncols) + " columns; the fixed scratch holds " + std::to_string(kScratchBytes) +
                    " (use fewer columns per call, or chfsi_apply)");
  if (t.has_proj && !ctx->scratch) return fail(ctx, CHFSI_EHIP, "fixed scratch unavailable: " + ctx->scratch_err);
  HIP_TRY(ctx, launch_fill(Y, t.M, ncols * cf, ld * cf, sp, ctx->stream));
  void* hP = nullptr;
  if (t.has_proj) {
    char* base = static_cast<char*>(ctx->scratch);
    hP = base + part_bytes;
    CHECK(nl_project(op, prec, X, ld, ncols, base, hP, ldhp));
  }
  const HxLaunch L = make_hx(op, prec, X, ld, nullptr, ld, Y, ld, ncols, 1.0, 0.0, 0.0, false, hP, ldhp);
  return launch_hx_cells(op, L, prec);
}

int chfsi_bounds(chfsi_op* op, int32_t steps, const void* v0, uint64_t seed, double* b_upper, double* lmin_est) {
  if (!op) return CHFSI_EINVAL;
  if (steps < 1 || steps > 1000) return fail(op->ctx, CHFSI_EINVAL, "steps must be in [1, 1000]");
  if (!b_upper) return fail(op->ctx, CHFSI_EINVAL, "null output");
  return do_bounds(op, steps, static_cast<const double*>(v0), nullptr, seed, b_upper, lmin_est);
}

int chfsi_filter(chfsi_op* op, void* X, int64_t ncols, int64_t ld, int32_t m, double a, double b, double aL,
                 int32_t prec, int32_t block) {
  if (!op) return CHFSI_EINVAL;
  CHECK(check_block(op, X, ncols, ld));
  if (!prec_valid_for(op, prec)) return fail(op->ctx, CHFSI_EINVAL, "precision does not match the operator");
  if (m < 1) return fail(op->ctx, CHFSI_EINVAL, "degree m must be >= 1");
  if (!(aL < a && a < b) || !std::isfinite(aL) || !std::isfinite(b))
    return fail(op->ctx, CHFSI_EINVAL, "need aL < a < b");
  return do_filter(op, X, ncols, ld, m, a, b, aL, prec, block);
}

int chfsi_orthonormalize(chfsi_op* op, void* X, int64_t ncols, int64_t ld, double* L_host) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  CHECK(check_block(op, X, ncols, ld));
  const int cf = op->t.cplx ? 2 : 1;
  void* X2;
  CHECK(ws_get(ctx, WS_X2, static_cast<size_t>(op->t.M) * ncols * 8 * cf, &X2));
  CHECK(cholgs(op, static_cast<double*>(X), ld, static_cast<double*>(X2), ncols, ncols, L_host));
  HIP_TRY(ctx, launch_convert(X, ld * cf, CHFSI_F64, X2, ncols * cf, CHFSI_F64, op->t.M, ncols * cf, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return 0;
}

int chfsi_rayleigh_ritz(chfsi_op* op, void* X, int64_t ncols, int64_t ld, double* theta, double* resid) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  CHECK(check_block(op, X, ncols, ld));
  if (!theta) return fail(ctx, CHFSI_EINVAL, "null theta");
  const int cf = op->t.cplx ? 2 : 1;
  void* X2;
  CHECK(ws_get(ctx, WS_X2, static_cast<size_t>(op->t.M) * ncols * 8 * cf, &X2));
  CHECK(rayleigh_ritz(op, static_cast<double*>(X), ld, static_cast<double*>(X2), ncols, ncols, theta, resid));
  HIP_TRY(ctx, launch_convert(X, ld * cf, CHFSI_F64, X2, ncols * cf, CHFSI_F64, op->t.M, ncols * cf, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return 0;
}

int chfsi_rayleigh_ritz_split(chfsi_op* op, void* X, int64_t ncols, int64_t ld, int32_t nfr, int32_t mixed,
                              double* theta, void* Psi_fr, int64_t ld_fr) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  CHECK(check_block(op, X, ncols, ld));
  if (!theta || !Psi_fr) return fail(ctx, CHFSI_EINVAL, "null theta or Psi_fr");
  if (nfr < 1 || nfr > ncols) return fail(ctx, CHFSI_EINVAL, "need 1 <= nfr <= ncols");
  if (ld_fr < nfr) return fail(ctx, CHFSI_EINVAL, "ld_fr < nfr");
  if (ncols > 46340) return fail(ctx, CHFSI_EINVAL, "ncols too large for the N x N workspace");
  return rrgep_split(op, static_cast<double*>(X), ld, ncols, nfr, mixed != 0, theta, static_cast<double*>(Psi_fr),
                     ld_fr);
}

int chfsi_pass(chfsi_op* op, const chfsi_params* prm, void* Xv, int64_t ld, double a, double b, double aL,
               double* theta, double* resid) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  if (!prm || !theta) return fail(ctx, CHFSI_EINVAL, "null argument");
  const int64_t N = static_cast<int64_t>(prm->nwanted) + prm->n_buf;
  if (prm->nwanted < 1 || prm->n_buf < 0) return fail(ctx, CHFSI_EINVAL, "nwanted >= 1, n_buf >= 0");
  CHECK(check_block(op, Xv, N, ld));
  if (prm->m < 1) return fail(ctx, CHFSI_EINVAL, "degree m must be >= 1");
  if (!prec_valid_for(op, prm->filter_prec)) return fail(ctx, CHFSI_EINVAL, "filter precision does not match");
  if (!(aL < a && a < b)) return fail(ctx, CHFSI_EINVAL, "need aL < a < b");
  const int cf = op->t.cplx ? 2 : 1;
  double* X = static_cast<double*>(Xv);
  void* X2v;
  CHECK(ws_get(ctx, WS_X2, static_cast<size_t>(op->t.M) * N * 8 * cf, &X2v));
  CHECK(do_filter(op, X, N, ld, prm->m, a, b, aL, prm->filter_prec, prm->block));
  CHECK(cholgs(op, X, ld, static_cast<double*>(X2v), N, N, nullptr));
  std::vector<double> r(N);
  CHECK(rayleigh_ritz(op, static_cast<double*>(X2v), N, X, ld, N, theta, r.data()));
  if (resid) std::memcpy(resid, r.data(), N * 8);
  return check_ritz(ctx, theta, r.data(), N, b);
}

int chfsi_fermi_level(const double* theta, int32_t n, const double* weights, double n_electrons, double kT,
                      double* mu, double* occ) {
  if (!theta || !mu || n < 1 || !(kT > 0.0) || !std::isfinite(kT)) return CHFSI_EINVAL;
  double wsum = 0.0, lo = theta[0], hi = theta[0];
  for (int32_t i = 0; i < n; ++i) {
    const double wi = weights ? weights[i] : 1.0;
    if (!std::isfinite(theta[i]) || !(wi >= 0.0)) return CHFSI_EINVAL;
    wsum += wi;
    lo = std::min(lo, theta[i]);
    hi = std::max(hi, theta[i]);
  }
  if (!(n_electrons > 0.0) || !(n_electrons < 2.0 * wsum)) return CHFSI_EINVAL;
  // f(e) = 1 / (1 + exp((e - mu) / kT)), written so that exp never overflows
  auto fermi = [kT](double e, double m) {
    const double x = (e - m) / kT;
    if (x > 0.0) {
      const double t = std::exp(-x);
      return t / (1.0 + t);
    }
    return 1.0 / (1.0 + std::exp(x));
  };
  auto count = [&](double m) {
    double c = 0.0;
    for (int32_t i = 0; i < n; ++i) c += (weights ? weights[i] : 1.0) * fermi(theta[i], m);
    return 2.0 * c;
  };
  // the count rises monotonically with mu: bisect to the width of a double
  lo -= 50.0 * kT;
  hi += 50.0 * kT;
  for (int it = 0; it < 2000 && hi - lo > 0.0; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count(mid) < n_electrons) lo = mid;
    else hi = mid;
  }
  *mu = 0.5 * (lo + hi);
  if (occ)
    for (int32_t i = 0; i < n; ++i) occ[i] = fermi(theta[i], *mu);
  return 0;
}

int chfsi_density(chfsi_op* op, const void* X, int64_t ncols, int64_t ld, const double* w, int32_t points,
                  int32_t accumulate, double* rho) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  CHECK(check_block(op, X, ncols, ld));
  if (!w || !rho) return fail(ctx, CHFSI_EINVAL, "null weights or output");
  if (points != CHFSI_RHO_NODES && points != CHFSI_RHO_GAUSS)
    return fail(ctx, CHFSI_EINVAL, "points must be CHFSI_RHO_NODES or CHFSI_RHO_GAUSS");
  for (int64_t i = 0; i < ncols; ++i)
    if (!std::isfinite(w[i])) return fail(ctx, CHFSI_EINVAL, "weights must be finite");
  const HostTables& t = op->t;
  const int cf = t.cplx ? 2 : 1;
  if (ncols * cf > (1LL << 30) || ld * cf > (1LL << 40)) return fail(ctx, CHFSI_EINVAL, "block too wide");
  void* dw;
  CHECK(ws_get(ctx, WS_DENS, static_cast<size_t>(ncols) * 8, &dw));
  HIP_TRY(ctx, hipMemcpyAsync(dw, w, static_cast<size_t>(ncols) * 8, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // w may be reused once the call returns
  DensityLaunch d{};
  d.X = static_cast<const double*>(X);
  d.ld = ld;
  d.ncols = static_cast<int>(ncols);
  d.cplx = t.cplx;
  d.w = static_cast<const double*>(dw);
  d.dscale = op->dscale;
  d.rho = rho;
  d.M = t.M;
  d.E = t.E;
  d.p = t.p;
  d.nc = t.ncell;
  d.points = points;
  d.accumulate = accumulate ? 1 : 0;
  d.interp = t.interp.data();
  HIP_TRY(ctx, launch_density(d, ctx->stream));
  return 0;
}

int chfsi_op_set_potential(chfsi_op* op, const double* V) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  if (!V) return fail(ctx, CHFSI_EINVAL, "null potential");
  if (op->astride != 0) return fail(ctx, CHFSI_EINVAL, "the operator integrates its potential per cell");
  const HostTables& t = op->t;
  const double k2 = 0.5 * (t.k[0] * t.k[0] + t.k[1] * t.k[1] + t.k[2] * t.k[2]);
  HIP_TRY(ctx, launch_convert(op->vdiag, 1, CHFSI_F64, V, 1, CHFSI_F64, t.M, 1, ctx->stream));
  if (k2 != 0.0) {
    void* one;
    CHECK(ws_get(ctx, WS_VEC, static_cast<size_t>(t.M) * 8, &one));
    std::vector<double> h(static_cast<size_t>(t.M), k2);
    HIP_TRY(ctx, hipMemcpyAsync(one, h.data(), h.size() * 8, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, launch_axpby(1.0, static_cast<double*>(one), 1.0, op->vdiag, t.M, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  return 0;
}

int chfsi_hartree(chfsi_op* op, const double* rho, double* vH, double tol, int32_t maxit, int32_t* iters,
                  double* relres) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  if (!rho || !vH) return fail(ctx, CHFSI_EINVAL, "null density or output");
  if (op->astride != 0) return fail(ctx, CHFSI_EINVAL, "the Hartree solve uses an operator with a nodal potential");
  if (!(tol > 0.0) || maxit < 1) return fail(ctx, CHFSI_EINVAL, "need tol > 0 and maxit >= 1");
  void* w;
  CHECK(ws_get(ctx, WS_SCF, static_cast<size_t>(op->t.M) * 6 * 8, &w));
  int it = 0;
  double rr = 0.0;
  CHECK(hartree_solve(op, rho, vH, tol, maxit, static_cast<double*>(w), &it, &rr));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (iters) *iters = it;
  if (relres) *relres = rr;
  return rr <= tol ? 0 : CHFSI_NOTCONV;
}

// The SCF loop over nk k-points of one mesh (nk = 1: chfsi_scf): operator,
// block and normalised weight of each k-point; the density, the Hartree
// potential and the mixing are shared, the eigensolver step runs per k-point
// and the Fermi level is taken over all k-points' Ritz values with their
// weights.
static int scf_loop(chfsi_ctx* ctx, int nk, chfsi_op* const* ops, void* const* Xvs, const int64_t* lds,
                    const double* wk, int32_t nwanted, int32_t n_buf, int32_t m, int32_t block, int32_t rr_mode,
                    double n_electrons, double kT, double beta, int32_t depth, double tol, int32_t maxit,
                    double* rho, double* const* thetas, double* mu_out, double* res_hist, int32_t* iters) {
  chfsi_op* op = ops[0];
  const HostTables& t = op->t;
  const int64_t N = static_cast<int64_t>(nwanted) + n_buf;
  for (int k = 0; k < nk; ++k) {
    const chfsi_op* o = ops[k];
    if (!o || o->ctx != ctx) return fail(ctx, CHFSI_EINVAL, "null operator, or one of another context");
    if (o->t.M != t.M || o->t.ncell != t.ncell || o->t.p != t.p || o->t.L != t.L)
      return fail(ctx, CHFSI_EINVAL, "the k-points of an SCF loop must share the mesh");
    if (o->astride != 0) return fail(ctx, CHFSI_EINVAL, "the SCF loop runs on operators with a nodal potential");
    CHECK(check_block(ops[k], Xvs[k], N, lds[k]));
    if (!thetas[k]) return fail(ctx, CHFSI_EINVAL, "null theta");
  }
  if (!rho) return fail(ctx, CHFSI_EINVAL, "null density");
  if (nwanted < 1 || n_buf < 0 || m < 1 || maxit < 1 || depth < 0 || depth > 16 || !(beta > 0.0) ||
      !(kT > 0.0) || !(tol > 0.0) || !(n_electrons > 0.0) || !(n_electrons < 2.0 * nwanted) || rr_mode < 0 ||
      rr_mode > 2)
    return fail(ctx, CHFSI_EINVAL, "bad SCF parameters");
  const int64_t M = t.M;
  hipStream_t st = ctx->stream;
  CHECK(scf_tables(op));
  const double* vext = op->scf_tab;
  const double* sqm = op->scf_tab + M;
  const double* mm = op->scf_tab + 2 * M;
  const int H = depth + 1;
  // work: CG 6 M, vH, V, rho_in, rho_out, F, weighted F, 2 H history, 2 depth differences
  const int64_t nvec = 6 + 6 + 2 * H + 2 * std::max(1, depth);
  void* wv;
  CHECK(ws_get(ctx, WS_SCF, static_cast<size_t>(M) * nvec * 8, &wv));
  double* w = static_cast<double*>(wv);
  double* cg = w;
  double* vh = w + 6 * M;
  double* V = vh + M;
  double* rin = V + M;
  double* rout = rin + M;
  double* F = rout + M;
  double* WF = F + M;
  std::vector<double*> xs(H), fs(H), dX(std::max(1, depth)), dF(std::max(1, depth));
  for (int i = 0; i < H; ++i) {
    xs[i] = WF + M + static_cast<int64_t>(i) * M;
    fs[i] = WF + M + static_cast<int64_t>(H + i) * M;
  }
  for (int i = 0; i < std::max(1, depth); ++i) {
    dX[i] = WF + M + static_cast<int64_t>(2 * H + i) * M;
    dF[i] = WF + M + static_cast<int64_t>(2 * H + std::max(1, depth) + i) * M;
  }
  HIP_TRY(ctx, launch_convert(rin, 1, CHFSI_F64, rho, 1, CHFSI_F64, M, 1, st));
  chfsi_params prm{};
  prm.nwanted = nwanted;
  prm.n_buf = n_buf;
  prm.m = m;
  prm.block = block > 0 ? block : static_cast<int32_t>(N);
  // per k-point: the real operator at Gamma, the complex Bloch operator H(k)
  // elsewhere (its density is real: |psi|^2 of the complex states)
  std::vector<std::vector<double>> th(nk, std::vector<double>(N));
  std::vector<double> f(nwanted), occ(static_cast<size_t>(nk) * nwanted), wfr, thall(occ.size()), wall(occ.size());
  int hist = 0, it = 0;
  bool conv = false;
  double mu = 0.0;
  // spectrum splitting (rr_mode 1: FP64, 2: mixed precision): the nfr
  // highest Ritz vectors of each step, the states below them being fully
  // occupied (chosen from the previous step's occupations)
  std::vector<int> nfr(nk, static_cast<int>(N));
  std::vector<double*> Pfr(nk, nullptr);
  std::vector<double> vhost(M), v0;   // effective potentials (host): this step's, the first step's
  std::vector<double> b0(nk, 0.0);    // Lanczos bounds of the first step's operators
  if (rr_mode > 0) {
    void* pv;
    const size_t per = static_cast<size_t>(M) * N * 2;   // doubles per k-point (complex room)
    CHECK(ws_get(ctx, WS_PFR, per * nk * 8, &pv));
    for (int k = 0; k < nk; ++k) Pfr[k] = static_cast<double*>(pv) + per * k;
  }
  for (it = 0; it < maxit; ++it) {
    // potential of the input density
    int cgit = 0;
    double cgr = 0.0;
    // from the previous step's potential after the first step
    CHECK(hartree_solve(op, rin, vh, 1e-10, 5000, cg, &cgit, &cgr, it > 0));
    HIP_TRY(ctx, launch_veff(vext, vh, rin, V, M, st));
    for (int k = 0; k < nk; ++k) CHECK(chfsi_op_set_potential(ops[k], V));
    // upper bound of the spectrum: Lanczos on the first step's operator;
    // later the potential only moves the diagonal, so by Weyl's inequality
    // lambda_max(H + dV) <= lambda_max(H) + max_j dV_j bounds it without
    // another Lanczos run
    HIP_TRY(ctx, hipMemcpyAsync(vhost.data(), V, M * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    double dmax = 0.0;
    if (it == 0) {
      for (int k = 0; k < nk; ++k) CHECK(do_bounds(ops[k], 20, nullptr, nullptr, 12345, &b0[k], nullptr));
      v0 = vhost;
    } else {
      for (int64_t j = 0; j < M; ++j) dmax = std::max(dmax, vhost[j] - v0[j]);
    }
    for (int k = 0; k < nk; ++k) {
      chfsi_op* opk = ops[k];
      void* Xv = Xvs[k];
      const int64_t ld = lds[k];
      std::vector<double>& thk = th[k];
      const int xprec = opk->t.cplx ? CHFSI_C128 : CHFSI_F64;
      prm.filter_prec = xprec;
      const double b = b0[k] + dmax;
      // eigensolver: the first step orthonormalises the start block and runs
      // four passes, later steps one pass from the previous subspace
      if (it == 0) {
        CHECK(chfsi_orthonormalize(opk, Xv, N, ld, nullptr));
        CHECK(chfsi_rayleigh_ritz(opk, Xv, N, ld, thk.data(), nullptr));
      }
      const bool split = rr_mode > 0 && it > 0;
      const int passes = it == 0 ? 4 : 1;
      for (int ps = 0; ps < passes; ++ps) {
        const double a = thk[N - 1], aL = thk[0];
        if (!(a < b)) return fail(ctx, CHFSI_EDIVERGE, "Ritz values above the spectrum bound");
        if (!split) {
          CHECK(chfsi_pass(opk, &prm, Xv, ld, a, b, aL, thk.data(), nullptr));
          continue;
        }
        // Algorithm 1's eigensolver step in the paper's form: the filter, then
        // Rayleigh-Ritz through the generalised problem with spectrum
        // splitting (Algorithm 2): X becomes the orthonormal basis Psi_o,
        // Pfr the nfr highest Ritz vectors
        CHECK(do_filter(opk, Xv, N, ld, m, a, b, aL, xprec, prm.block));
        CHECK(rrgep_split(opk, static_cast<double*>(Xv), ld, N, nfr[k], rr_mode == 2, thk.data(), Pfr[k], nfr[k]));
        CHECK(check_ritz(ctx, thk.data(), nullptr, N, b));
      }
    }
    // occupations over all k-points (weights w_k), and the output density
    for (int k = 0; k < nk; ++k)
      for (int i = 0; i < nwanted; ++i) {
        thall[static_cast<size_t>(k) * nwanted + i] = th[k][i];
        wall[static_cast<size_t>(k) * nwanted + i] = wk[k];
      }
    CHECK(chfsi_fermi_level(thall.data(), nk * nwanted, wall.data(), n_electrons, kT, &mu, occ.data()));
    const bool split = rr_mode > 0 && it > 0;
    for (int k = 0; k < nk; ++k) {
      const double* ok = occ.data() + static_cast<size_t>(k) * nwanted;
      if (!split) {
        for (int i = 0; i < nwanted; ++i) f[i] = 2.0 * wk[k] * ok[i];
        CHECK(chfsi_density(ops[k], Xvs[k], nwanted, lds[k], f.data(), CHFSI_RHO_NODES, k > 0, rout));
      } else {
        // Algorithm 3's split form: every basis vector counted fully
        // occupied, then the nfr highest Ritz vectors corrected by
        // 2 (f_i - 1) (buffer states: f_i = 0); exact when f_i = 1 below
        // the split
        std::vector<double> two(N, 2.0 * wk[k]);
        CHECK(chfsi_density(ops[k], Xvs[k], N, lds[k], two.data(), CHFSI_RHO_NODES, k > 0, rout));
        wfr.assign(nfr[k], 0.0);
        for (int j = 0; j < nfr[k]; ++j) {
          const int64_t i = N - nfr[k] + j;
          wfr[j] = 2.0 * wk[k] * ((i < nwanted ? ok[i] : 0.0) - 1.0);
        }
        CHECK(chfsi_density(ops[k], Pfr[k], nfr[k], nfr[k], wfr.data(), CHFSI_RHO_NODES, 1, rout));
      }
      if (rr_mode > 0) {
        // next split: all states whose vacancy 1 - f exceeds 1e-14, plus two
        int full = 0;
        while (full < nwanted && 1.0 - ok[full] <= 1e-14) ++full;
        nfr[k] = static_cast<int>(std::min<int64_t>(N, N - full + 2));
      }
    }
    // residual F = rho_out - rho_in in the M-weighted norm
    HIP_TRY(ctx, launch_convert(F, 1, CHFSI_F64, rout, 1, CHFSI_F64, M, 1, st));
    HIP_TRY(ctx, launch_axpby(-1.0, rin, 1.0, F, M, st));
    HIP_TRY(ctx, launch_emul(F, mm, WF, M, st));
    double r2 = 0.0;
    CHECK(dot_host(ctx, F, WF, M, &r2));
    const double res = std::sqrt(std::max(r2, 0.0));
    if (res_hist) res_hist[it] = res;
    if (res < tol) {
      conv = true;
      ++it;
      break;
    }
    // Anderson mixing over the last `depth` differences
    if (hist == H) {
      std::rotate(xs.begin(), xs.begin() + 1, xs.end());
      std::rotate(fs.begin(), fs.begin() + 1, fs.end());
      --hist;
    }
    HIP_TRY(ctx, launch_convert(xs[hist], 1, CHFSI_F64, rin, 1, CHFSI_F64, M, 1, st));
    HIP_TRY(ctx, launch_convert(fs[hist], 1, CHFSI_F64, F, 1, CHFSI_F64, M, 1, st));
    ++hist;
    const int nd = hist - 1;
    std::vector<double> g(nd, 0.0);
    if (nd > 0) {
      for (int i = 0; i < nd; ++i) {
        HIP_TRY(ctx, launch_convert(dX[i], 1, CHFSI_F64, xs[i + 1], 1, CHFSI_F64, M, 1, st));
        HIP_TRY(ctx, launch_axpby(-1.0, xs[i], 1.0, dX[i], M, st));
        HIP_TRY(ctx, launch_convert(dF[i], 1, CHFSI_F64, fs[i + 1], 1, CHFSI_F64, M, 1, st));
        HIP_TRY(ctx, launch_axpby(-1.0, fs[i], 1.0, dF[i], M, st));
      }
      std::vector<double> A(static_cast<size_t>(nd) * nd), rv(nd);
      for (int i = 0; i < nd; ++i) {
        HIP_TRY(ctx, launch_emul(dF[i], mm, cg, M, st));   // M-weighted copy
        CHECK(dot_host(ctx, cg, F, M, &rv[i]));
        for (int j = 0; j <= i; ++j) {
          CHECK(dot_host(ctx, cg, dF[j], M, &A[static_cast<size_t>(i) * nd + j]));
          A[static_cast<size_t>(j) * nd + i] = A[static_cast<size_t>(i) * nd + j];
        }
      }
      // least squares by Gaussian elimination with a tiny ridge
      double tr = 0.0;
      for (int i = 0; i < nd; ++i) tr += A[static_cast<size_t>(i) * nd + i];
      for (int i = 0; i < nd; ++i) A[static_cast<size_t>(i) * nd + i] += 1e-12 * tr / nd;
      g = rv;
      for (int c = 0; c < nd; ++c) {
        int pr = c;
        for (int r = c + 1; r < nd; ++r)
          if (std::fabs(A[static_cast<size_t>(r) * nd + c]) > std::fabs(A[static_cast<size_t>(pr) * nd + c])) pr = r;
        if (pr != c) {
          for (int k = 0; k < nd; ++k) std::swap(A[static_cast<size_t>(c) * nd + k], A[static_cast<size_t>(pr) * nd + k]);
          std::swap(g[c], g[pr]);
        }
        const double piv = A[static_cast<size_t>(c) * nd + c];
        if (piv == 0.0) continue;
        for (int r = c + 1; r < nd; ++r) {
          const double fct = A[static_cast<size_t>(r) * nd + c] / piv;
          for (int k = c; k < nd; ++k) A[static_cast<size_t>(r) * nd + k] -= fct * A[static_cast<size_t>(c) * nd + k];
          g[r] -= fct * g[c];
        }
      }
      for (int c = nd - 1; c >= 0; --c) {
        double sacc = g[c];
        for (int k = c + 1; k < nd; ++k) sacc -= A[static_cast<size_t>(c) * nd + k] * g[k];
        const double piv = A[static_cast<size_t>(c) * nd + c];
        g[c] = piv != 0.0 ? sacc / piv : 0.0;
      }
    }
    // rho_in <- (x - dX g) + beta (F - dF g)
    for (int i = 0; i < nd; ++i) {
      HIP_TRY(ctx, launch_axpby(-g[i], dX[i], 1.0, rin, M, st));
      HIP_TRY(ctx, launch_axpby(-g[i], dF[i], 1.0, F, M, st));
    }
    HIP_TRY(ctx, launch_axpby(beta, F, 1.0, rin, M, st));
  }
  HIP_TRY(ctx, launch_convert(rho, 1, CHFSI_F64, conv ? rout : rin, 1, CHFSI_F64, M, 1, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  for (int k = 0; k < nk; ++k) std::memcpy(thetas[k], th[k].data(), N * 8);
  if (mu_out) *mu_out = mu;
  if (iters) *iters = it;
  return conv ? 0 : CHFSI_NOTCONV;
}

int chfsi_scf(chfsi_op* op, void* Xv, int64_t ld, int32_t nwanted, int32_t n_buf, int32_t m, int32_t block,
              int32_t rr_mode, double n_electrons, double kT, double beta, int32_t depth, double tol, int32_t maxit,
              double* rho, double* theta, double* mu_out, double* res_hist, int32_t* iters) {
  if (!op) return CHFSI_EINVAL;
  const double one = 1.0;
  double* const thetas[1] = {theta};
  return scf_loop(op->ctx, 1, &op, &Xv, &ld, &one, nwanted, n_buf, m, block, rr_mode, n_electrons, kT, beta, depth,
                  tol, maxit, rho, thetas, mu_out, res_hist, iters);
}

int chfsi_scf_kpoints(chfsi_ctx* ctx, int32_t nk, chfsi_op* const* ops, void* const* X, const int64_t* ld,
                      const double* weights, int32_t nwanted, int32_t n_buf, int32_t m, int32_t block,
                      int32_t rr_mode, double n_electrons, double kT, double beta, int32_t depth, double tol,
                      int32_t maxit, double* rho, double* const* theta, double* mu_out, double* res_hist,
                      int32_t* iters) {
  if (!ctx) return CHFSI_EINVAL;
  if (nk < 1 || !ops || !X || !ld || !theta) return fail(ctx, CHFSI_EINVAL, "null argument or nk < 1");
  std::vector<double> w(nk, 1.0 / nk);
  if (weights) {
    double sum = 0.0;
    for (int k = 0; k < nk; ++k) {
      if (!(weights[k] >= 0.0) || !std::isfinite(weights[k])) return fail(ctx, CHFSI_EINVAL, "bad k-point weight");
      sum += weights[k];
    }
    if (!(sum > 0.0)) return fail(ctx, CHFSI_EINVAL, "k-point weights sum to zero");
    for (int k = 0; k < nk; ++k) w[k] = weights[k] / sum;
  }
  return scf_loop(ctx, nk, ops, X, ld, w.data(), nwanted, n_buf, m, block, rr_mode, n_electrons, kT, beta, depth,
                  tol, maxit, rho, theta, mu_out, res_hist, iters);
}

int chfsi_set_timing(chfsi_ctx* ctx, int32_t enable) {
  if (!ctx) return CHFSI_EINVAL;
  ctx->timing = enable != 0;
  return 0;
}

int chfsi_set_deterministic(chfsi_ctx* ctx, int32_t enable) {
  if (!ctx) return CHFSI_EINVAL;
  if (enable) {
    // colour classes of the live operators now (one cell per side: none; such
    // an operator is refused at its first H~.X while the mode is on)
    for (const void* o : ctx->live_ops) {
      chfsi_op* op = static_cast<chfsi_op*>(const_cast<void*>(o));
      if (op->t.ncell >= 2) CHECK(build_colours(op));
    }
  }
  ctx->deterministic = enable != 0;
  return 0;
}

int chfsi_kernel_time(chfsi_ctx* ctx, double* total_ms, int64_t* launches, double* flops, int32_t reset) {
  if (!ctx) return CHFSI_EINVAL;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (size_t i = 0; i < ctx->pending.size(); ++i) {
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->pending[i].first, ctx->pending[i].second));
    ctx->t_ms += ms;
    ctx->t_flops += ctx->pending_flops[i];
    ctx->t_launches += 1;
    (void)hipEventDestroy(ctx->pending[i].first);
    (void)hipEventDestroy(ctx->pending[i].second);
  }
  ctx->pending.clear();
  ctx->pending_flops.clear();
  if (total_ms) *total_ms = ctx->t_ms;
  if (launches) *launches = ctx->t_launches;
  if (flops) *flops = ctx->t_flops;
  if (reset) {
    ctx->t_ms = 0.0;
    ctx->t_flops = 0.0;
    ctx->t_launches = 0;
  }
  return 0;
}

int chfsi_solve(chfsi_op* op, const chfsi_params* prm, void* Xv, int64_t ld, double* theta, double* resid,
                chfsi_stats* stats) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* ctx = op->ctx;
  if (!prm || !theta) return fail(ctx, CHFSI_EINVAL, "null argument");
  const HostTables& t = op->t;
  const int64_t N = static_cast<int64_t>(prm->nwanted) + prm->n_buf;
  if (prm->nwanted < 1 || prm->n_buf < 0) return fail(ctx, CHFSI_EINVAL, "nwanted >= 1, n_buf >= 0");
  CHECK(check_block(op, Xv, N, ld));
  if (prm->m < 1) return fail(ctx, CHFSI_EINVAL, "degree m must be >= 1");
  if (!prec_valid_for(op, prm->filter_prec)) return fail(ctx, CHFSI_EINVAL, "filter precision does not match");
  if (prm->fixed_passes <= 0 && !(prm->tol > 0.0)) return fail(ctx, CHFSI_EINVAL, "need fixed_passes or tol");
  if (prm->hist_len < 0) return fail(ctx, CHFSI_EINVAL, "hist_len must be >= 0");
  const int cf = t.cplx ? 2 : 1;
  hipEvent_t ev[8];
  for (auto& e : ev) HIP_TRY(ctx, hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { for (int i = 0; i < 8; ++i) (void)hipEventDestroy(e[i]); }
  } guard{ev};
  chfsi_stats st;
  std::memset(&st, 0, sizeof(st));
  st.final_prec = prm->filter_prec;
  HIP_TRY(ctx, hipEventRecord(ev[0], ctx->stream));
  double b = prm->b_upper;
  if (!(b > 0.0)) {
    const int steps = prm->lanczos_steps > 0 ? prm->lanczos_steps : 20;
    double lmin;
    CHECK(do_bounds(op, steps, nullptr, prm->lanczos_v0, prm->seed, &b, &lmin));
    st.hx_columns += steps;
  }
  HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
  st.t_bounds = 0.0;
  double* X = static_cast<double*>(Xv);
  void* X2v;
  CHECK(ws_get(ctx, WS_X2, static_cast<size_t>(t.M) * N * 8 * cf, &X2v));
  double* X2 = static_cast<double*>(X2v);
  std::vector<double> th(N), r(N);
  // initial CholGS + RR: X -> X2 (orthonormal) -> X (Ritz vectors).  A start
  // block that is rank deficient to working precision (repeated or dependent
  // columns) is repaired once: its columns from the first dependent one on
  // are redrawn N(0, 1) from the seed, and the CholGS is repeated.
  int64_t bad = -1;
  const int rc0 = cholgs(op, X, ld, X2, N, N, nullptr, &bad);
  if (rc0 == CHFSI_ECHOL && bad >= 0 && bad < N) {
    const int64_t nr = (N - bad) * cf;
    std::vector<double> h(static_cast<size_t>(t.M) * nr);
    SplitMix g{prm->seed ^ 0x7265647261770000ULL};
    for (auto& x : h) x = g.normal();
    HIP_TRY(ctx, hipMemcpy2DAsync(X + bad * cf, ld * cf * 8, h.data(), nr * 8, nr * 8, t.M, hipMemcpyHostToDevice,
                                  ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    st.redrawn_columns = static_cast<int32_t>(N - bad);
    CHECK(cholgs(op, X, ld, X2, N, N, nullptr));
  } else if (rc0 < 0) {
    return rc0;
  }
  CHECK(rayleigh_ritz(op, X2, N, X, ld, N, th.data(), r.data()));
  st.hx_columns += N;
  auto max_r = [&]() {
    double m = 0.0;
    for (int i = 0; i < prm->nwanted; ++i) m = std::max(m, r[i]);
    return m;
  };
  std::vector<double> rhist{max_r()};
  if (prm->hist_len > 0) {
    HIP_TRY(ctx, hipEventRecord(ev[5], ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(ev[5]));
    record_hist(*prm, 0, event_ms(ev[0], ev[5]), rhist[0], -1, th.data(), N);
  }
  const int limit = prm->fixed_passes > 0 ? prm->fixed_passes : (prm->max_passes > 0 ? prm->max_passes : 100);
  int passes = 0;
  int fprec = prm->filter_prec;
  double a = th[N - 1], aL = th[0];
  while (passes < limit) {
    if (prm->fixed_passes <= 0 && max_r() <= prm->tol) break;
    a = th[N - 1];
    aL = th[0];
    if (!(aL < a && a < b)) return fail(ctx, CHFSI_EDIVERGE, "filter interval collapsed (b below the Ritz values?)");
    HIP_TRY(ctx, hipEventRecord(ev[2], ctx->stream));
    CHECK(do_filter(op, X, N, ld, prm->m, a, b, aL, fprec, prm->block));
    HIP_TRY(ctx, hipEventRecord(ev[3], ctx->stream));
    CHECK(cholgs(op, X, ld, X2, N, N, nullptr));
    HIP_TRY(ctx, hipEventRecord(ev[4], ctx->stream));
    CHECK(rayleigh_ritz(op, X2, N, X, ld, N, th.data(), r.data()));
    HIP_TRY(ctx, hipEventRecord(ev[5], ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(ev[5]));
    st.t_filter += event_ms(ev[2], ev[3]);
    st.t_cholgs += event_ms(ev[3], ev[4]);
    st.t_rr += event_ms(ev[4], ev[5]);
    st.hx_columns += static_cast<int64_t>(N) * prm->m + N;
    ++passes;
    CHECK(check_ritz(ctx, th.data(), r.data(), N, b));
    rhist.push_back(max_r());
    record_hist(*prm, passes, event_ms(ev[0], ev[5]), rhist.back(), fprec, th.data(), N);
    st.final_prec = fprec;
    if (prm->prec_switch) {
      const int np = next_prec(fprec, rhist.data(), static_cast<int>(rhist.size()) - 1, b);
      if (np != fprec) ++st.prec_changes;
      fprec = np;
    }
  }
  HIP_TRY(ctx, hipEventRecord(ev[6], ctx->stream));
  HIP_TRY(ctx, hipEventSynchronize(ev[6]));
  st.t_bounds = event_ms(ev[0], ev[1]);
  st.t_total = event_ms(ev[0], ev[6]);
  st.passes = passes;
  st.b_upper = b;
  st.a_last = a;
  st.aL_last = aL;
  st.max_resid = max_r();
  st.hx_flops = static_cast<double>(st.hx_columns) * 2.0 * t.mcell * t.mcell * t.E * (t.cplx ? 4.0 : 1.0);
  std::memcpy(theta, th.data(), N * 8);
  if (resid) std::memcpy(resid, r.data(), N * 8);
  if (stats) *stats = st;
  if (prm->fixed_passes <= 0 && st.max_resid > prm->tol) {
    ctx->err = "tolerance not met";
    return CHFSI_NOTCONV;
  }
  return 0;
}

int chfsi_filter_batched(chfsi_ctx* ctx, int32_t n, chfsi_op* const* ops, void* const* X, const int64_t* ncols,
                         const int64_t* ld, int32_t m, const double* a, const double* b, const double* aL,
                         int32_t prec, int32_t block, int32_t use_graph) {
  if (!ctx) return CHFSI_EINVAL;
  if (n < 1 || !ops || !X || !ncols || !ld || !a || !b || !aL) return fail(ctx, CHFSI_EINVAL, "null argument");
  if (m < 1) return fail(ctx, CHFSI_EINVAL, "degree m must be >= 1");
  std::vector<BItem> items(n);
  for (int q = 0; q < n; ++q) {
    if (!ops[q]) return fail(ctx, CHFSI_EINVAL, "null operator");
    CHECK(check_block(ops[q], X[q], ncols[q], ld[q]));
    items[q] = BItem{ops[q], static_cast<double*>(X[q]), ncols[q], ld[q], a[q], b[q], aL[q]};
  }
  return batched_filter(ctx, items, m, prec, block, use_graph != 0);
}

}  // extern "C"

namespace {

// CholGS and Rayleigh-Ritz of several problems whose blocks have at most
// kSmallMaxN columns, with the N x N steps of all problems in one launch each
// (small_cholinv_kernel, small_eigh_kernel: one workgroup per problem) and
// two host synchronisations in all (the Cholesky flags, then the Ritz values,
// residual partials and eigensolve flags).  The O(M N) and O(M N^2) steps
// (Gram products, rotations, H~ X_o, residuals) are launched problem by
// problem on the context's stream.  Problem q = idx[k]: X[q] (ld[q]) holds
// the block on entry and the Ritz vectors on exit; th[q], r[q] (N[q]) the
// Ritz values and residual norms.  Same results as cholgs() + rayleigh_ritz()
// per problem.
int subspace_small_batched(chfsi_ctx* ctx, const std::vector<int>& idx, chfsi_op* const* ops, void* const* Xv,
                           const int64_t* ld, const std::vector<int64_t>& N, std::vector<std::vector<double>>& th,
                           std::vector<std::vector<double>>& r) {
  const int na = static_cast<int>(idx.size());
  if (na == 0) return 0;
  // per-problem device storage: X_o, W = H~ X_o, H Psi (M x N each), S, H^,
  // Z (N x N, real view of Z for complex: 2N x 2N), eigenvalues, residual
  // partials; then the pointer / dimension tables and the flags
  std::vector<size_t> oX2(na), oW(na), oHP(na), oS(na), oH(na), oZ(na), oD(na), oR(na);
  size_t tot = 0;
  auto take = [&](size_t bytes) { const size_t at = tot; tot += align256(bytes); return at; };
  for (int k = 0; k < na; ++k) {
    const int q = idx[k];
    const chfsi_op* op = ops[q];
    const size_t cf = op->t.cplx ? 2 : 1;
    const size_t mn = static_cast<size_t>(op->t.M) * N[q] * cf * 8;
    const size_t nn = static_cast<size_t>(N[q]) * N[q] * cf * 8;
    oX2[k] = take(mn);
    oW[k] = take(mn);
    oHP[k] = take(mn);
    oS[k] = take(nn);
    oH[k] = take(nn);
    oZ[k] = take(nn * cf);
    oD[k] = take(static_cast<size_t>(N[q]) * 8);
    oR[k] = take(resid_partial_count(op->t.M, static_cast<int>(N[q])) * 8);
  }
  const size_t oTab = take(static_cast<size_t>(na) * (3 * sizeof(double*) + sizeof(int)));
  const size_t oInfo = take(static_cast<size_t>(na) * 2 * sizeof(int));
  void* wsv;
  CHECK(ws_get(ctx, WS_SUBB, tot, &wsv));
  char* base = static_cast<char*>(wsv);
  auto at = [&](size_t o) { return reinterpret_cast<double*>(base + o); };
  int* dinfo = reinterpret_cast<int*>(base + oInfo);   // [0, na): Cholesky, [na, 2 na): eigensolve
  // device tables: S pointers, H^ pointers, eigenvalue pointers, dimensions
  std::vector<char> htab(static_cast<size_t>(na) * (3 * sizeof(double*) + sizeof(int)));
  double** hS = reinterpret_cast<double**>(htab.data());
  double** hH = hS + na;
  double** hD = hH + na;
  int* hdim = reinterpret_cast<int*>(hD + na);
  int nmax = 0;
  for (int k = 0; k < na; ++k) {
    hS[k] = at(oS[k]);
    hH[k] = at(oH[k]);
    hD[k] = at(oD[k]);
    hdim[k] = static_cast<int>(N[idx[k]]);
    nmax = std::max(nmax, hdim[k]);
  }
  if (nmax > kSmallMaxN) return fail(ctx, CHFSI_EINVAL, "batched small subspace step: block too wide");
  // the table travels through the pinned staging buffer (stream-ordered after
  // any earlier use of it, which the host has synchronised before rewriting)
  void* pin;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  CHECK(pinned_get(ctx, htab.size(), &pin));
  std::memcpy(pin, htab.data(), htab.size());
  char* dtab = base + oTab;
  HIP_TRY(ctx, hipMemcpyAsync(dtab, pin, htab.size(), hipMemcpyHostToDevice, ctx->stream));
  SmallBatch sb;
  sb.dims = reinterpret_cast<const int*>(dtab + static_cast<size_t>(na) * 3 * sizeof(double*));
  // 1. S_q = X_q^H X_q; all Cholesky factors and inverses in one launch
  for (int k = 0; k < na; ++k) {
    const int q = idx[k];
    double* S = at(oS[k]);
    CHECK(gram(ops[q], static_cast<const double*>(Xv[q]), ld[q], static_cast<const double*>(Xv[q]), ld[q], N[q],
               &S));
  }
  sb.mats = reinterpret_cast<double* const*>(dtab);
  sb.info = dinfo;
  const bool cplx = ops[idx[0]]->t.cplx;
  HIP_TRY(ctx, launch_small_cholinv(sb, na, cplx, ctx->stream));
  std::vector<int> hinfo(2 * static_cast<size_t>(na));
  HIP_TRY(ctx, hipMemcpyAsync(hinfo.data(), dinfo, na * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < na; ++k)
    if (hinfo[k] != 0)
      return fail(ctx, CHFSI_ECHOL, "overlap matrix of problem " + std::to_string(idx[k]) +
                                        " is not positive definite (leading minor " + std::to_string(hinfo[k]) + ")");
  // 2. X_o = X L^-H, W = H~ X_o, H^ = X_o^H W
  for (int k = 0; k < na; ++k) {
    const int q = idx[k];
    chfsi_op* op = ops[q];
    const int cf = op->t.cplx ? 2 : 1;
    const int64_t Nq = N[q];
    const int n1 = static_cast<int>(Nq);
    double* S = at(oS[k]);
    const double* Z = S;
    int64_t ldz = Nq;
    if (op->t.cplx) {
      HIP_TRY(ctx, launch_expand_complex(S, n1, n1, 1, at(oZ[k]), ctx->stream));
      Z = at(oZ[k]);
      ldz = 2 * Nq;
    } else {
      HIP_TRY(ctx, launch_zero_strict_lower(S, n1, Nq, ctx->stream));
    }
    double* X2 = at(oX2[k]);
    HIP_TRY(ctx, launch_rotate(static_cast<const double*>(Xv[q]), ld[q] * cf, Z, ldz, X2, Nq * cf, op->t.M,
                               static_cast<int>(Nq * cf), static_cast<int>(Nq * cf), true, ctx->stream));
    const int prec = op->t.cplx ? CHFSI_C128 : CHFSI_F64;
    double* W = at(oW[k]);
    HIP_TRY(ctx, launch_fill(W, op->t.M, Nq * cf, Nq * cf, prec, ctx->stream));
    CHECK(hx_step(op, prec, X2, Nq, nullptr, 0, W, Nq, Nq, 1.0, 0.0, 0.0, false));
    double* Hh = at(oH[k]);
    CHECK(gram(op, X2, Nq, W, Nq, Nq, &Hh));
  }
  // 3. all eigensolves in one launch
  sb.mats = reinterpret_cast<double* const*>(dtab + static_cast<size_t>(na) * sizeof(double*));
  sb.evals = reinterpret_cast<double* const*>(dtab + static_cast<size_t>(na) * 2 * sizeof(double*));
  sb.info = dinfo + na;
  HIP_TRY(ctx, launch_small_eigh(sb, na, cplx, ctx->stream));
  // 4. Psi = X_o Q, H Psi = W Q, residual partials; results to the host
  std::vector<int> nch(na);
  size_t hbytes = 0;
  std::vector<size_t> hoR(na), hoD(na);
  for (int k = 0; k < na; ++k) {
    const int q = idx[k];
    hoR[k] = hbytes;
    hbytes += resid_partial_count(ops[q]->t.M, static_cast<int>(N[q])) * 8;
    hoD[k] = hbytes;
    hbytes += static_cast<size_t>(N[q]) * 8;
  }
  for (int k = 0; k < na; ++k) {
    const int q = idx[k];
    chfsi_op* op = ops[q];
    const int cf = op->t.cplx ? 2 : 1;
    const int64_t Nq = N[q];
    const int n1 = static_cast<int>(Nq);
    double* Hh = at(oH[k]);
    double* Zb = at(oZ[k]);
    int64_t ldz;
    if (op->t.cplx) {
      HIP_TRY(ctx, launch_expand_complex(Hh, n1, n1, 2, Zb, ctx->stream));
      ldz = 2 * Nq;
    } else {
      HIP_TRY(ctx, launch_transpose(Hh, Zb, n1, ctx->stream));
      ldz = Nq;
    }
    double* X2 = at(oX2[k]);
    double* W = at(oW[k]);
    double* HP = at(oHP[k]);
    HIP_TRY(ctx, launch_rotate(X2, Nq * cf, Zb, ldz, static_cast<double*>(Xv[q]), ld[q] * cf, op->t.M,
                               static_cast<int>(Nq * cf), static_cast<int>(Nq * cf), false, ctx->stream));
    HIP_TRY(ctx, launch_rotate(W, Nq * cf, Zb, ldz, HP, Nq * cf, op->t.M, static_cast<int>(Nq * cf),
                               static_cast<int>(Nq * cf), false, ctx->stream));
    HIP_TRY(ctx, launch_resid(HP, Nq, static_cast<double*>(Xv[q]), ld[q], at(oD[k]), op->t.M, n1, op->t.cplx,
                              at(oR[k]), &nch[k], ctx->stream));
  }
  void* hres;
  CHECK(pinned_get(ctx, hbytes, &hres));   // the table copy above has completed (synchronised in step 1)
  char* hb = static_cast<char*>(hres);
  for (int k = 0; k < na; ++k) {
    const int q = idx[k];
    HIP_TRY(ctx, hipMemcpyAsync(hb + hoR[k], at(oR[k]), static_cast<size_t>(nch[k]) * N[q] * 8,
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(hb + hoD[k], at(oD[k]), static_cast<size_t>(N[q]) * 8, hipMemcpyDeviceToHost,
                                ctx->stream));
  }
  HIP_TRY(ctx, hipMemcpyAsync(hinfo.data() + na, dinfo + na, na * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < na; ++k) {
    const int q = idx[k];
    if (hinfo[na + k] != 0)
      return fail(ctx, CHFSI_EHIP, "projected eigensolve of problem " + std::to_string(q) + " did not converge");
    const double* rp = reinterpret_cast<const double*>(hb + hoR[k]);
    const double* D = reinterpret_cast<const double*>(hb + hoD[k]);
    for (int64_t j = 0; j < N[q]; ++j) {
      double sum = 0.0;
      for (int c = 0; c < nch[k]; ++c) sum += rp[static_cast<size_t>(c) * N[q] + j];
      r[q][j] = std::sqrt(sum);
      th[q][j] = D[j];
    }
  }
  return 0;
}

}  // namespace

extern "C" {

int chfsi_solve_batched(chfsi_ctx* ctx, int32_t n, chfsi_op* const* ops, const chfsi_params* params,
                        void* const* Xv, const int64_t* ld, double* const* theta, double* const* resid,
                        chfsi_stats* stats, int32_t use_graph) {
  if (!ctx) return CHFSI_EINVAL;
  if (n < 1 || !ops || !params || !Xv || !ld || !theta) return fail(ctx, CHFSI_EINVAL, "null argument");
  const int m = params[0].m;
  const int prec = params[0].filter_prec;
  const int64_t block = params[0].block;
  std::vector<int64_t> N(n);
  for (int q = 0; q < n; ++q) {
    const chfsi_params& pr = params[q];
    if (!ops[q] || !theta[q]) return fail(ctx, CHFSI_EINVAL, "null operator or output");
    if (ops[q]->ctx != ctx) return fail(ctx, CHFSI_EINVAL, "operators must share the context");
    if (pr.m != m || pr.filter_prec != prec || pr.block != block)
      return fail(ctx, CHFSI_EINVAL, "m, block and filter_prec must be equal across the batch");
    if (pr.nwanted < 1 || pr.n_buf < 0 || pr.m < 1) return fail(ctx, CHFSI_EINVAL, "bad parameters");
    if (pr.fixed_passes <= 0 && !(pr.tol > 0.0)) return fail(ctx, CHFSI_EINVAL, "need fixed_passes or tol");
    if (pr.prec_switch) return fail(ctx, CHFSI_EINVAL, "prec_switch is not available in the batched solve");
    if (pr.hist_len < 0) return fail(ctx, CHFSI_EINVAL, "hist_len must be >= 0");
    N[q] = static_cast<int64_t>(pr.nwanted) + pr.n_buf;
    CHECK(check_block(ops[q], Xv[q], N[q], ld[q]));
    if (!prec_valid_for(ops[q], prec)) return fail(ctx, CHFSI_EINVAL, "filter precision does not match");
  }
  hipEvent_t e0, e1, es;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  HIP_TRY(ctx, hipEventCreate(&es));
  struct G3 {
    hipEvent_t a, b, c;
    ~G3() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); (void)hipEventDestroy(c); }
  } guard{e0, e1, es};
  HIP_TRY(ctx, hipEventRecord(es, ctx->stream));
  std::vector<double> bq(n), aq(n), aLq(n);
  std::vector<std::vector<double>> th(n), r(n);
  std::vector<int> passes(n, 0);
  std::vector<char> done(n, 0);
  std::vector<double> tfilt(n, 0.0), tcg(n, 0.0), trr(n, 0.0);
  auto maxr_of = [&](int q) {
    double mr = 0.0;
    for (int i = 0; i < params[q].nwanted; ++i) mr = std::max(mr, r[q][i]);
    return mr;
  };
  // every block of at most kSmallMaxN columns: the CholGS and Rayleigh-Ritz
  // steps of all problems together (one launch per N x N step)
  bool all_small = true;
  for (int q = 0; q < n; ++q) all_small = all_small && N[q] <= kSmallMaxN;
  std::vector<int> all(n);
  for (int q = 0; q < n; ++q) {
    chfsi_op* op = ops[q];
    const chfsi_params& pr = params[q];
    double b = pr.b_upper;
    if (!(b > 0.0)) {
      double lmin;
      CHECK(do_bounds(op, pr.lanczos_steps > 0 ? pr.lanczos_steps : 20, nullptr, pr.lanczos_v0, pr.seed, &b, &lmin));
    }
    bq[q] = b;
    th[q].assign(N[q], 0.0);
    r[q].assign(N[q], 0.0);
    all[q] = q;
    if (all_small) continue;
    const int cf = op->t.cplx ? 2 : 1;
    void* X2v;
    CHECK(ws_get(ctx, WS_X2, static_cast<size_t>(op->t.M) * N[q] * 8 * cf, &X2v));
    CHECK(cholgs(op, static_cast<double*>(Xv[q]), ld[q], static_cast<double*>(X2v), N[q], N[q], nullptr));
    CHECK(rayleigh_ritz(op, static_cast<double*>(X2v), N[q], static_cast<double*>(Xv[q]), ld[q], N[q],
                        th[q].data(), r[q].data()));
    if (pr.hist_len > 0) {
      HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
      HIP_TRY(ctx, hipEventSynchronize(e1));
      record_hist(pr, 0, event_ms(es, e1), maxr_of(q), -1, th[q].data(), N[q]);
    }
  }
  if (all_small) {
    CHECK(subspace_small_batched(ctx, all, ops, Xv, ld, N, th, r));
    HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(e1));
    for (int q = 0; q < n; ++q)
      if (params[q].hist_len > 0) record_hist(params[q], 0, event_ms(es, e1), maxr_of(q), -1, th[q].data(), N[q]);
  }
  auto converged = [&](int q) {
    const chfsi_params& pr = params[q];
    const int limit = pr.fixed_passes > 0 ? pr.fixed_passes : (pr.max_passes > 0 ? pr.max_passes : 100);
    if (passes[q] >= limit) return true;
    if (pr.fixed_passes > 0) return false;
    double mr = 0.0;
    for (int i = 0; i < pr.nwanted; ++i) mr = std::max(mr, r[q][i]);
    return mr <= pr.tol;
  };
  for (;;) {
    std::vector<BItem> items;
    std::vector<int> idx;
    for (int q = 0; q < n; ++q) {
      if (done[q] || converged(q)) { done[q] = 1; continue; }
      aq[q] = th[q][N[q] - 1];
      aLq[q] = th[q][0];
      if (!(aLq[q] < aq[q] && aq[q] < bq[q])) return fail(ctx, CHFSI_EDIVERGE, "filter interval collapsed");
      items.push_back(BItem{ops[q], static_cast<double*>(Xv[q]), N[q], ld[q], aq[q], bq[q], aLq[q]});
      idx.push_back(q);
    }
    if (items.empty()) break;
    HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
    CHECK(batched_filter(ctx, items, m, prec, block, use_graph != 0));
    HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(e1));
    const double tf = event_ms(e0, e1);
    if (all_small) {
      // the subspace step of all active problems together; its time is
      // shared evenly among them in the statistics
      HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
      CHECK(subspace_small_batched(ctx, idx, ops, Xv, ld, N, th, r));
      HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
      HIP_TRY(ctx, hipEventSynchronize(e1));
      const double ts = event_ms(e0, e1) / static_cast<double>(idx.size());
      for (int q : idx) {
        trr[q] += ts;
        tfilt[q] += tf;
        ++passes[q];
        CHECK(check_ritz(ctx, th[q].data(), r[q].data(), N[q], bq[q]));
        record_hist(params[q], passes[q], event_ms(es, e1), maxr_of(q), prec, th[q].data(), N[q]);
      }
      continue;
    }
    for (int q : idx) {
      chfsi_op* op = ops[q];
      const int cf = op->t.cplx ? 2 : 1;
      void* X2v;
      CHECK(ws_get(ctx, WS_X2, static_cast<size_t>(op->t.M) * N[q] * 8 * cf, &X2v));
      HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
      CHECK(cholgs(op, static_cast<double*>(Xv[q]), ld[q], static_cast<double*>(X2v), N[q], N[q], nullptr));
      CHECK(rayleigh_ritz(op, static_cast<double*>(X2v), N[q], static_cast<double*>(Xv[q]), ld[q], N[q],
                          th[q].data(), r[q].data()));
      HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
      HIP_TRY(ctx, hipEventSynchronize(e1));
      trr[q] += event_ms(e0, e1);
      tfilt[q] += tf;
      ++passes[q];
      CHECK(check_ritz(ctx, th[q].data(), r[q].data(), N[q], bq[q]));
      record_hist(params[q], passes[q], event_ms(es, e1), maxr_of(q), prec, th[q].data(), N[q]);
    }
  }
  drop_graph(ctx);
  int rc = 0;
  for (int q = 0; q < n; ++q) {
    std::memcpy(theta[q], th[q].data(), N[q] * 8);
    if (resid && resid[q]) std::memcpy(resid[q], r[q].data(), N[q] * 8);
    const double mr = maxr_of(q);
    if (stats) {
      chfsi_stats& st = stats[q];
      std::memset(&st, 0, sizeof(st));
      st.passes = passes[q];
      st.final_prec = prec;
      st.t_filter = tfilt[q];
      st.t_rr = trr[q];
      st.b_upper = bq[q];
      st.a_last = aq[q];
      st.aL_last = aLq[q];
      st.max_resid = mr;
      st.hx_columns = static_cast<int64_t>(passes[q]) * (N[q] * m + N[q]) + N[q];
      st.hx_flops = static_cast<double>(passes[q]) * hx_flops(ops[q], N[q] * m + N[q]);
    }
    if (params[q].fixed_passes <= 0 && mr > params[q].tol) rc = CHFSI_NOTCONV;
  }
  if (rc == CHFSI_NOTCONV) ctx->err = "tolerance not met for at least one problem";
  return rc;
}

int chfsi_autotune(chfsi_ctx* ctx, const char* cache_json, int32_t p, int32_t prec, int32_t block) {
  if (!ctx) return CHFSI_EINVAL;
  if (p < kMinOrder || p > kMaxOrder) return fail(ctx, CHFSI_EINVAL, "order p must be in [2, 7]");
  if (prec != CHFSI_F64 && prec != CHFSI_F32 && prec != CHFSI_C128 && prec != CHFSI_C64)
    return fail(ctx, CHFSI_EINVAL, "autotune supports F64, F32, C128, C64");
  if (block < 1 || block > 1024) return fail(ctx, CHFSI_EINVAL, "block must be in [1, 1024]");
  if (cache_json) CHECK(load_tuning_file(ctx, cache_json));
  // synthetic batch: 4 uneven empty periodic boxes of order p (h = 2 bohr)
  const bool cplx = (prec == CHFSI_C128 || prec == CHFSI_C64);
  const int ncs[4] = {6, 8, 9, 10};
  std::vector<chfsi_op*> ops;
  std::vector<void*> bufs;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(ctx->stream);
    for (auto* o : ops) chfsi_op_destroy(o);
    for (void* b : bufs) (void)hipFree(b);
  };
  int rc = 0;
  std::vector<BItem> items;
  for (int i = 0; i < 4 && rc == 0; ++i) {
    chfsi_system sys;
    std::memset(&sys, 0, sizeof(sys));
    sys.L = 2.0 * ncs[i];
    sys.ncell = ncs[i];
    sys.p = p;
    if (cplx) { sys.k[0] = 0.1; sys.k[1] = 0.05; sys.k[2] = -0.07; }
    chfsi_op* op = nullptr;
    rc = chfsi_op_build(ctx, &sys, &op);
    if (rc < 0) break;
    ops.push_back(op);
    const int cf = cplx ? 2 : 1;
    void* X = nullptr;
    const size_t bytes = static_cast<size_t>(op->t.M) * block * 8 * cf;
    if (hipMalloc(&X, bytes) != hipSuccess) { rc = fail(ctx, CHFSI_ENOMEM, "autotune allocation failed"); break; }
    bufs.push_back(X);
    if (hipMemsetAsync(X, 0, bytes, ctx->stream) != hipSuccess) { rc = fail(ctx, CHFSI_EHIP, "memset failed"); break; }
    items.push_back(BItem{op, static_cast<double*>(X), block, block, 1.0, 4.0, -1.0});
  }
  if (rc < 0) { cleanup(); return rc; }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  chfsi_ctx::Tuning best;
  best.ms = 1e300;
  const int m = 4;
  for (int nt : {64, 32})
  for (int g = 0; g <= 4 && rc == 0; ++g)
    for (int cont = 1; cont >= 0 && rc == 0; --cont) {
      if (g == 0 && cont == 1) continue;  // one item per workgroup: assignment is moot
      chfsi_ctx::Tuning t;
      t.grid_per_cu = g;
      t.contiguous = cont;
      t.col_tile = nt;
      rc = batched_filter(ctx, items, m, prec, block, false, &t);  // warm-up
      if (rc < 0) break;
      (void)hipEventRecord(e0, ctx->stream);
      rc = batched_filter(ctx, items, m, prec, block, false, &t);
      if (rc < 0) break;
      (void)hipEventRecord(e1, ctx->stream);
      (void)hipEventSynchronize(e1);
      t.ms = event_ms(e0, e1);
      if (t.ms < best.ms) best = t;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cleanup();
  if (rc < 0) return rc;
  ctx->tuning[tune_key(p, prec, block)] = best;
  if (cache_json) CHECK(save_tuning_file(ctx, cache_json));
  return 0;
}

int chfsi_load_tuning(chfsi_ctx* ctx, const char* cache_json) {
  if (!ctx || !cache_json) return CHFSI_EINVAL;
  return load_tuning_file(ctx, cache_json);
}

int chfsi_get_tuning(chfsi_ctx* ctx, int32_t p, int32_t prec, int32_t block, int32_t* grid_per_cu,
                     int32_t* contiguous, int32_t* col_tile, double* ms) {
  if (!ctx) return CHFSI_EINVAL;
  const chfsi_ctx::Tuning t = tuning_for(ctx, p, prec, block);
  if (grid_per_cu) *grid_per_cu = t.grid_per_cu;
  if (contiguous) *contiguous = t.contiguous;
  if (col_tile) *col_tile = t.col_tile;
  if (ms) *ms = t.ms;
  return 0;
}

}  // extern "C"
