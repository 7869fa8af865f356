// Internal declarations shared by the host driver and the HIP kernels of
// libchfsi.  Not part of the public ABI (include/chfsi.h).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/chfsi.h"

namespace chfsi {

// Orders with compiled cell kernels.
constexpr int kMinOrder = 2;
constexpr int kMaxOrder = 7;

inline int mcell_of(int p) { return (p + 1) * (p + 1) * (p + 1); }
// Cell rows/k padded to a multiple of 16 (MFMA row tiles and 4-wide k steps).
inline int mpad_of(int p) { return (mcell_of(p) + 15) / 16 * 16; }

// Host-side tables of one operator (everything the kernels read).
struct HostTables {
  int p = 0, ncell = 0, n = 0;
  int64_t M = 0, E = 0;
  int mcell = 0, mpad = 0;
  bool cplx = false;
  double L = 0.0, h = 0.0, k[3] = {0, 0, 0};
  std::vector<double> x1d;          // n node coordinates along one axis
  std::vector<double> cell_re;      // mcell x mcell
  std::vector<double> cell_im;      // mcell x mcell (complex only)
  std::vector<double> dscale;       // per node M^-1/2 (M)
  std::vector<double> interp;       // (p+1) x (p+1): interp[q*(p+1)+a] = l_a(g_q)
  std::vector<double> K1d, M1d;     // 1D stiffness and consistent mass, (p+1) x (p+1)
  std::vector<double> vdiag;        // V + |k|^2/2 (M)
  int natoms = 0;
  bool has_proj = false;
  std::vector<double> hcoef;        // 4 * natoms couplings
  // atom-major projector node lists: for atom a, entries
  // [atom_ptr[a], atom_ptr[a+1]) of (node, 4 values c~ (x2 if complex)).
  std::vector<int64_t> atom_ptr;
  std::vector<int32_t> atom_node;
  std::vector<double> atom_val;     // per entry 4 (real) or 8 (re,im x 4)
  // (cell, atom) pairs sorted by cell, with the cell-local projector matrix
  // (mcell x 4, split by node multiplicity) in MFMA operand layout.
  std::vector<int32_t> pair_ptr;    // E + 1
  std::vector<int32_t> pair_atom;   // npairs
  std::vector<double> pair_re;      // npairs * (mpad/16) * 64
  std::vector<double> pair_im;      // complex only
  std::vector<double> atoms;        // natoms x 8: x, y, z, Z, s, h_s, h_p, 0
};

// n-point Gauss-Legendre nodes and weights on [-1, 1] (op_build.cpp).
void gauss_legendre_rule(int n, std::vector<double>& x, std::vector<double>& w);

// Builds the tables on the host (op_build.cpp).  Returns "" or an error text.
std::string build_tables(const chfsi_system& sys, HostTables& t);

// Swizzles a row-major mcell x mcell matrix into MFMA A-operand layout:
// out[(rt * ks_count + ks) * 64 + lane] = A[rt*16 + lane%16][ks*4 + lane/16].
void swizzle_cell_matrix(const double* A, int mcell, int mpad, double* out);
// bf16 (round to nearest even) operand order of v_mfma_f32_16x16x32_bf16, rows
// and k padded to a multiple of 32:
// out[((rt * ks_count + ks) * 64 + lane) * 8 + j] = A[rt*16 + lane%16][ks*32 + 8*(lane/16) + j]
int mpad32_of(int p);
void swizzle_cell_matrix_bf16(const double* A, int mcell, uint16_t* out);
uint16_t bf16_rne(float x);

// ---- kernel launchers (kernels_hx.hip, kernels_dense.hip) -----------------

struct HxLaunch {
  int p, nc;                       // order, cells per side
  int ncols;                       // real columns (2x complex columns)
  bool cplx;
  const void* A;                   // swizzled real part
  const void* Ai;                  // swizzled imaginary part (complex)
  const double* vdiag;             // V + |k|^2/2
  const void* Xk; int64_t ldx;     // X_k (real view)
  const void* Xp; int64_t ldp;     // X_{k-1} (nullable)
  void* T; int64_t ldt;            // accumulation target
  bool zero_prev;                  // owners write 0 into Xp after reading it
  double alpha, c, beta;
  // nonlocal (nullable when no projectors)
  const int32_t* pair_ptr; const int32_t* pair_atom;
  const void* pair_re; const void* pair_im;
  const void* hP; int64_t ldhp;    // scaled projector coefficients (real view)
  const void* Abf = nullptr;       // bf16 cell matrix in 16x16x32 operand order
  int64_t astride = 0;             // per-cell real matrices: elements per cell (0: shared)
  int ncu = 0;                     // compute units (persistent launches)
  int nt = 64;                     // columns per work item: 64, or 32 (not for BF16)
  // deterministic assembly: launch over one colour class of cells only
  // (device array of ncell cell ids, no two sharing a node); null: all cells
  const int32_t* cells = nullptr;
  int ncell = 0;
};

// prec: CHFSI_F64 / F32 / BF16 (real), C128 / C64 (complex, data real view).
hipError_t launch_cell_hx(const HxLaunch& a, int prec, hipStream_t s);

// Many problems of the same order and precision in one persistent launch.
// descs: device array of nprob packed kernel argument blocks (pack_hx_desc);
// item_off: device array of nprob + 1 item offsets (items of problem q are
// its E_q x ceil(ncols_q / nt) (cell, column tile) pairs).
struct HxBatch {
  int p;
  int nt = 64;     // columns per work item: 64 or 32
  const void* descs;
  const int64_t* item_off;
  int nprob;
  int grid;        // persistent workgroups
  int contiguous;  // 1: contiguous item range per workgroup, 0: strided
  int one_per_item = 0;  // grid equals the number of items: one item per workgroup
};
size_t hx_desc_bytes(int prec);
void pack_hx_desc(const HxLaunch& L, int prec, void* out);
hipError_t launch_cell_hx_batched(const HxBatch& b, int prec, hipStream_t s);

struct NlLaunch {
  int natoms;
  bool cplx;
  int ncols;                        // complex or real columns (logical)
  const int64_t* atom_ptr; const int32_t* atom_node; const double* atom_val;
  const int32_t* chunk_atom; const int64_t* chunk_begin; int nchunks;
  const int32_t* atom_chunk_ptr;
  const double* hcoef;
  const void* X; int64_t ldx;       // logical ld (complex entries for complex)
  void* partial;                    // nchunks x 4 x ldhp (real view)
  void* hP; int64_t ldhp;           // natoms*4 x ldhp (real view)
};
hipError_t launch_nl_project(const NlLaunch& a, int prec, hipStream_t s);

// The projection of nprob operators' blocks in two launches (batched filter):
// descs = device array of nprob NlLaunch; chunk_off / row_off = device
// arrays of nprob + 1 offsets of the problems' chunks and of their
// (atom, component) rows; max_col_tiles = max ceil(ncols / 64) and
// max_row_blocks = max ceil(ldhp / 256) over the problems.
struct NlBatch {
  const void* descs;
  const int64_t* chunk_off;
  const int64_t* row_off;
  int nprob;
  int64_t total_chunks, total_rows;
  int max_col_tiles, max_row_blocks;
};
hipError_t launch_nl_project_batched(const NlBatch& b, int prec, hipStream_t s);

// Size of the fixed device scratch of chfsi_apply_noalloc() (kernels_nl.hip),
// and its device address on the current device (call with that device
// current; each device has its own copy).
constexpr size_t kScratchBytes = size_t(64) << 20;
hipError_t scratch_address(void** out);

// Electron density (kernels_density.hip).  points 0: at the nodes (M
// values); 1: at the (p+1)^3 Gauss points of every cell (E x (p+1)^3).
struct DensityLaunch {
  const double* X; int64_t ld;      // logical ld (complex entries for complex)
  int ncols;                        // logical columns
  bool cplx;
  const double* w;                  // device, ncols weights
  const double* dscale;             // device, M^-1/2 per node
  double* rho;
  int64_t M, E;
  int p, nc;
  int points, accumulate;
  const double* interp;             // host, (p+1) x (p+1)
};
hipError_t launch_density(const DensityLaunch& d, hipStream_t s);

// Per-cell local potential by Gauss quadrature (kernels_dhm.hip).
// Vw[e * nq + q] = V(x_q^e) w_q |J| for the (p+1)^3 Gauss points of every cell.
hipError_t launch_gauss_potential(const double* atoms, int natoms, double L, int nc, int p, const double* gq,
                                  const double* gw, double* Vw, hipStream_t s);
// Ae (E x mpad^2, A-operand order) = Ash + D_i D_k Kloc_e[pair(i, k)].
hipError_t launch_assemble_cell_matrices(const double* Ash, const double* Kloc, int64_t msym, const double* Dl,
                                         int mcell, int mpad, int64_t E, double* Ae, hipStream_t s);

// SCF loop helpers (kernels_scf.hip), n values each.
hipError_t launch_hartree_rhs(const double* rho, double rho_bar, const double* sqm, double* b, int64_t n,
                              hipStream_t s);
hipError_t launch_ediv(const double* x, const double* d, double* y, int64_t n, hipStream_t s);
hipError_t launch_emul(const double* x, const double* d, double* y, int64_t n, hipStream_t s);
hipError_t launch_veff(const double* vext, const double* vh, const double* rho, double* V, int64_t n,
                       hipStream_t s);
// One preconditioned CG iteration after q = A p: with the device scalars
// sc (6 values: r.z, p.q, r.r, z.n, new r.z, n.n) it updates u, r, z (Jacobi,
// then projected off the null vector nv) and p, and stores r.r in hist[it].
// part (nullable, 5 x 256 values): the dot products' block partials are
// stored there and summed in a fixed order instead of added atomically
hipError_t launch_cg_iteration(double* u, double* r, double* z, double* p, const double* q, const double* kd,
                               const double* nv, double* sc, double* hist, int it, int64_t n, hipStream_t s,
                               double* part = nullptr);
// q += D K D u on the structured mesh by sum factorisation (K1, M1: the 1D
// stiffness and consistent mass, host, (p+1)^2 values each)
// (cells: the ncell cells of one colour class, no two sharing a node; null:
// every cell)
hipError_t launch_stiffness(const double* u, const double* dscale, double* q, int p, int nc, const double* K1,
                            const double* M1, hipStream_t s, const int32_t* cells = nullptr, int ncell = 0);

// Elementwise helpers on row-major blocks (real view).
hipError_t launch_fill(void* dst, int64_t rows, int64_t cols, int64_t ld, int prec, hipStream_t s);
// dst (type dprec) <- src (type sprec), rows x cols (real view)
hipError_t launch_convert(void* dst, int64_t ldd, int dprec, const void* src, int64_t lds, int sprec,
                          int64_t rows, int64_t cols, hipStream_t s);

// Dense FP64 kernels on real views.
// Lower-triangular Gram G = X^T Y (n x n, real view) -> partial buffers then
// reduced into G (row-major, ldg), upper triangle mirrored.
size_t gram_partial_bytes(int64_t M, int n, int64_t ld);
// X / Y may point offx / offy columns into their rows (a column slice of a
// block whose rows hold ldx / ldy values); offx + n <= ldx, offy + n <= ldy.
hipError_t launch_gram(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t M, int n,
                       double* partial, double* G, int64_t ldg, hipStream_t s, int64_t offx = 0,
                       int64_t offy = 0);
// the same product on FP32 data in FP32 arithmetic (per row chunk; the chunk
// partials are summed in FP64)
hipError_t launch_gram(const float* X, int64_t ldx, const float* Y, int64_t ldy, int64_t M, int n,
                       double* partial, double* G, int64_t ldg, hipStream_t s, int64_t offx = 0,
                       int64_t offy = 0);
// C = X Z, X: M x K (ldx), Z: K x N2 row-major (ldz); upper = Z upper-triangular.
hipError_t launch_rotate(const double* X, int64_t ldx, const double* Z, int64_t ldz, double* C,
                         int64_t ldc, int64_t M, int K, int N2, bool upper, hipStream_t s);
hipError_t launch_rotate(const float* X, int64_t ldx, const float* Z, int64_t ldz, float* C,
                         int64_t ldc, int64_t M, int K, int N2, bool upper, hipStream_t s);
// Residual column sums: partial[chunk][j] = sum_rows |HX[r][j] - th[j] X[r][j]|^2
// (complex: j indexes complex columns, data interleaved).
size_t resid_partial_count(int64_t M, int ncols);
hipError_t launch_resid(const double* HX, int64_t ldh, const double* X, int64_t ldx,
                        const double* theta, int64_t M, int ncols, bool cplx, double* partial,
                        int* nchunks_out, hipStream_t s);
// dot partial sums of two real-view vectors of length n: partial[block]
int dot_blocks();
hipError_t launch_dot(const double* x, const double* y, int64_t n, double* partial, hipStream_t s);
// y = a*x + b*y over n reals
hipError_t launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
// small matrix helpers (n x n)
hipError_t launch_transpose(const double* in, double* out, int n, hipStream_t s);
hipError_t launch_zero_strict_lower(double* A, int n, int64_t lda, hipStream_t s);
// out (cols x rows, ldo) = in^T for row-major in (rows x cols, ldi)
hipError_t launch_transpose_rect(const double* in, int64_t ldi, int rows, int cols, double* out, int64_t ldo,
                                 hipStream_t s);
// Zo (n x n FP32) = Z without its diagonal, d = diag(Z) (FP64)
hipError_t launch_split_diag(const double* Z, int64_t ldz, int n, float* Zo, double* d, hipStream_t s);
// X[r][j] = C[r][j] + d[j] X[r][j], C FP32, M x n
hipError_t launch_add_scaled_cols(const float* C, int64_t ldc, const double* d, double* X, int64_t ldx, int64_t M,
                                  int n, hipStream_t s);
// S[i][j] = G[max(i,j)][min(i,j)] (real symmetric from the lower Gram tiles)
hipError_t launch_sym_from_lower(const double* G, int64_t ldg, double* S, int n, hipStream_t s);
// complex Hermitian S (n x n column-major interleaved) from the real-view Gram
hipError_t launch_gram_combine_complex(const double* G2, int64_t ldg2, double* S, int n, hipStream_t s);
// ---- small dense kernels (kernels_small.hip), one workgroup per matrix ----
// Every matrix is column-major n x n (n <= kSmallMaxN), complex interleaved.
// Matrix q of a launch of `count` workgroups is mats[q] (n = dims[q],
// eigenvalues to evals[q]) when the device arrays are given, else the single
// matrix mat0 (n0, ev0).  info[q] (device) = 0 on success.
// cholinv: lower triangle of S -> L^-1 with S = L L^H (info k + 1 at a
// non-positive k-th pivot, S then unchanged).  eigh: lower triangle of H ->
// eigenvectors (column j for the j-th), eigenvalues ascending (info 1: no
// convergence).
constexpr int kSmallMaxN = 64;
struct SmallBatch {
  double* const* mats = nullptr;
  const int* dims = nullptr;
  double* const* evals = nullptr;
  double* mat0 = nullptr;
  int n0 = 0;
  double* ev0 = nullptr;
  int* info = nullptr;
};
hipError_t launch_small_cholinv(const SmallBatch& b, int count, bool cplx, hipStream_t s);
hipError_t launch_small_eigh(const SmallBatch& b, int count, bool cplx, hipStream_t s);

// real 2n1 x 2n2 expansion of a complex matrix: mode 0 row-major Z, mode 1
// column-major L^-1 -> Z = L^-H (upper), mode 2 column-major Q -> Z = Q
hipError_t launch_expand_complex(const double* Z, int n1, int n2, int mode, double* Z2, hipStream_t s);

// ---- warm-start network kernels (kernels_mlp.hip), FP32 -------------------
// C = epi(A W) with A (M x K, lda), W read as W[k * swk + n * swn], N <= 128.
// mode 0: + bias (nullable); 1: tanh(. + bias); 2: D0 - A W; 3: (A W) * (1 - D0^2).
hipError_t mlp_gemm(const float* A, int64_t lda, const float* W, int64_t swk, int64_t swn, float* C, int64_t ldc,
                    int64_t M, int K, int N, int mode, const float* bias, const float* D0, int64_t ldd, hipStream_t s);
// G = A^T B (KA x KB <= 128 x 128, ldg) with a deterministic split over rows.
size_t mlp_gram_partial_bytes(int64_t M);
hipError_t mlp_gram(const float* A, int64_t lda, int KA, const float* B, int64_t ldb, int KB, int64_t M, float* part,
                    float* G, int ldg, hipStream_t s);
size_t mlp_colsum_partial_bytes(int64_t M, int N);
hipError_t mlp_colsum(const float* A, int64_t lda, int N, int64_t M, double* part, float* out, hipStream_t s);
int mlp_dot_blocks();
hipError_t mlp_dot(const float* x, const float* y, int64_t n, double* part, hipStream_t s);
hipError_t mlp_loss_small(const float* G, int n, double sY, float* D, double* out, hipStream_t s);
hipError_t mlp_combine(float c1, const float* R, float c2, const float* Y, float c3, const float* YD, float* dY,
                       int64_t n, hipStream_t s);
hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                    int t, hipStream_t s);
hipError_t mlp_normalize(const float* F, const float* mean, const float* stdv, float* Fn, int64_t M, int din,
                         hipStream_t s);
hipError_t launch_features(const double* x1d, int n, double L, const double* atoms, int natoms, int kimg, double eta,
                           double rcut, float* F, hipStream_t s);

}  // namespace chfsi
