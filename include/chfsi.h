/*
 * chfsi.h -- C ABI of libchfsi: Chebyshev-filtered subspace iteration on the
 * spectral finite-element Kohn-Sham Hamiltonian, on one AMD Instinct MI355X
 * (gfx950).
 *
 * The method is the eigensolver of DFT-FE 1.0 (Das, Motamarri, Subramanian,
 * Rogers, Gavini, arXiv 2203.07820): the Chebyshev filter of Section 3.1
 * (Eq. chebyfilter), whose every step is the cell-wise product H~.X of
 * Section 4.3 (Eq. celldgemm, Algorithm 4 for the nonlocal part), followed by
 * the Cholesky-Gram-Schmidt orthonormalisation and Rayleigh-Ritz steps of
 * Algorithm 2.  H~ = M^-1/2 H M^-1/2 is the Loewdin-transformed discrete
 * Hamiltonian of Section 2.3 (discrete H^loc and H^nl equations, GLL-lumped
 * overlap M).
 *
 * Conventions
 * -----------
 * - Every function returns an int status: 0 on success, a negative error
 *   code, or a positive warning.  The text of the last error is available
 *   from chfsi_last_error().  No C++ exception crosses this boundary.
 * - Arrays documented "device" are device pointers on the context's GPU
 *   (for instance torch.Tensor.data_ptr() of a CUDA tensor); all other
 *   array arguments are host pointers.
 * - Blocks of vectors are row-major M x ld arrays: row j holds the values of
 *   node j for all columns (all B values of one node are contiguous, the
 *   node-major layout of Section 4.3), ld >= ncols.  Complex data
 *   (CHFSI_C128 / CHFSI_C64) is interleaved (re, im) and ld counts complex
 *   entries.
 * - Ownership: the caller owns every array it passes.  The library never
 *   frees a caller pointer and does not keep it after the call returns,
 *   except while work it enqueued on the context's stream is in flight.
 *   Operators own their device tables until chfsi_op_destroy().  The context
 *   owns its scratch memory, which only grows, until chfsi_ctx_destroy().
 * - Work is enqueued on the stream given to chfsi_ctx_create().  Functions
 *   documented "synchronous" wait for that stream before returning.
 * - A context and its operators are not thread-safe: use one thread per
 *   context.
 * - Invalid arguments (null required pointers, ld < ncols, ncols > M, an
 *   order outside [2, 7], a precision that does not match the operator,
 *   a > b or aL >= a for the filter) return CHFSI_EINVAL before any work is
 *   enqueued.
 */
#ifndef CHFSI_H
#define CHFSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CHFSI_OK         0
#define CHFSI_NOTCONV    1   /* warning: tolerance not met; results valid   */
#define CHFSI_EINVAL    (-1) /* invalid argument                            */
#define CHFSI_ENOMEM    (-2) /* device allocation failed                    */
#define CHFSI_EHIP      (-3) /* HIP runtime or library error                */
#define CHFSI_ECHOL     (-4) /* overlap matrix not positive definite        */
#define CHFSI_EDIVERGE  (-5) /* non-finite values, or a Ritz value above the
                                 upper bound b (b below lambda_max)          */

/* ---- arithmetic / storage precision ------------------------------------ */
typedef enum {
  CHFSI_F64  = 0, /* real double                                           */
  CHFSI_F32  = 1, /* real float                                            */
  CHFSI_BF16 = 2, /* real: float storage, cell products on bf16-rounded
                     inputs (round to nearest even) with float accumulation */
  CHFSI_C128 = 3, /* complex double (Bloch k != 0)                          */
  CHFSI_C64  = 4  /* complex float                                         */
} chfsi_prec;

typedef struct chfsi_ctx chfsi_ctx;
typedef struct chfsi_op chfsi_op;
typedef struct chfsi_mlp chfsi_mlp;

/* A periodic cube [0, L)^3 of ncell^3 hexahedral cells of order p, with
 * Gaussian atoms (Section 2.3 discretisation; synthetic stand-ins for the
 * pseudopotential atoms of Section 5).
 *   V(x)   = sum_a sum_images -Z_a exp(-|x - R_a - nL|^2 / (2 s_a^2)),
 *            image terms within 10 s_a;
 *   chi_s  = n_s exp(-r^2/(2 w^2)), chi_p,alpha = n_p r_alpha exp(...),
 *            unit L2 norm, zero beyond r = 6 w, couplings h_s and h_p
 *            (separable form of Eq. nlps / nonlocalHamDiscrete);
 *   k      = Bloch vector (Eq. contEigenBZ); k = 0 gives a real operator.
 * pos has 3*natoms entries (x, y, z per atom).  w, h_s, h_p are read only
 * when has_proj != 0.  All arrays are host arrays copied by the call. */
typedef struct {
  double L;
  int32_t ncell;
  int32_t p;
  int32_t natoms;
  int32_t has_proj;
  const double* pos;
  const double* Z;
  const double* s;
  const double* w;
  const double* h_s;
  const double* h_p;
  double k[3];
} chfsi_system;

/* Parameters of chfsi_solve().
 *   nwanted        N: number of wanted eigenpairs;
 *   n_buf          extra buffer columns filtered with the wanted ones
 *                  (X has N + n_buf columns);
 *   m              Chebyshev degree;
 *   block          column block B filtered at a time (Section 4.3 blocked
 *                  H~.X);
 *   fixed_passes   > 0: run exactly this many passes; else iterate until
 *                  max_{i<N} r_i <= tol or max_passes;
 *   filter_prec    arithmetic of the filter: F64, F32 or BF16 for a real
 *                  operator, C128 or C64 for a complex one.  Orthonormalis-
 *                  ation, Rayleigh-Ritz and residuals are always FP64;
 *   lanczos_steps  steps of the Lanczos run that gives the upper bound b;
 *   b_upper        > 0: use this bound instead of running Lanczos;
 *   lanczos_v0     optional host vector (M real or 2M interleaved complex
 *                  values) that starts Lanczos; NULL draws one from seed;
 *   seed           seed of the library's own generator (splitmix64 +
 *                  Box-Muller) when lanczos_v0 is NULL;
 *   prec_switch    1: mixed-precision schedule.  After each pass the filter
 *                  precision is raised one level (BF16 -> F32 -> F64,
 *                  C64 -> C128) once r = max_{i<N} r_i has reached the
 *                  level's rounding floor, r <= 4 u b (u = 2^-8 for BF16,
 *                  2^-24 for F32 and C64; b the upper bound), or once r has
 *                  grown in two passes in a row.  0: the precision stays;
 *   hist_len       entries available in each non-NULL history array below;
 *                  entry 0 describes the initial Rayleigh-Ritz, entry i the
 *                  state after pass i; passes beyond hist_len - 1 are not
 *                  recorded;
 *   hist_time_ms   host, nullable: milliseconds from the start of the solve
 *                  (bound included) to the end of that pass;
 *   hist_max_resid host, nullable: max_{i<N} r_i after that pass;
 *   hist_prec      host, nullable: filter precision of that pass (-1 for
 *                  entry 0);
 *   hist_theta     host, nullable: hist_len x (N + n_buf) Ritz values. */
typedef struct {
  int32_t nwanted;
  int32_t n_buf;
  int32_t m;
  int32_t block;
  int32_t fixed_passes;
  int32_t max_passes;
  double tol;
  int32_t filter_prec;
  int32_t lanczos_steps;
  double b_upper;
  const double* lanczos_v0;
  uint64_t seed;
  int32_t prec_switch;
  int32_t hist_len;
  double* hist_time_ms;
  double* hist_max_resid;
  int32_t* hist_prec;
  double* hist_theta;
} chfsi_params;

/* Timings (milliseconds, from HIP events on the context stream) and counts
 * filled by chfsi_solve(). */
typedef struct {
  double t_bounds;
  double t_filter;
  double t_cholgs;
  double t_rr;
  double t_total;
  int32_t passes;
  int64_t hx_columns;       /* number of single-column H~ applications    */
  double hx_flops;          /* algorithmic cell-product flops (padding excluded) */
  double b_upper;           /* bound used                                 */
  double a_last, aL_last;   /* filter interval of the last pass           */
  double max_resid;         /* max_{i<N} r_i after the last pass          */
  int32_t final_prec;       /* filter precision of the last pass          */
  int32_t prec_changes;     /* passes after which the precision was raised */
  int32_t redrawn_columns;  /* start-block columns redrawn because the block
                               was rank deficient (chfsi_solve; 0: none)   */
} chfsi_stats;

/* ---- context ------------------------------------------------------------ */
/* Create a context on HIP device `device`; all work goes to `hip_stream`
 * (a hipStream_t; NULL means the legacy default stream). */
int chfsi_ctx_create(chfsi_ctx** out, int device, void* hip_stream);
/* Destroys the context.  It keeps a registry of the operators and networks
 * built on it; while any of them is alive the call returns CHFSI_EINVAL,
 * leaves the context untouched and usable, and names the count in
 * chfsi_last_error(ctx): destroy them first.  NULL is a no-op. */
int chfsi_ctx_destroy(chfsi_ctx* ctx);
/* Text of the last error of this context ("" if none).  Valid until the next
 * call on the context.  ctx may be NULL (errors of chfsi_ctx_create). */
const char* chfsi_last_error(const chfsi_ctx* ctx);
/* Wait for all work enqueued on the context stream. */
int chfsi_sync(chfsi_ctx* ctx);
/* Library version string. */
const char* chfsi_version(void);
/* sizeof of chfsi_system, chfsi_params and chfsi_stats as this library was
 * built, so that a binding can check its own struct layouts (any pointer may
 * be NULL).  Needs no device. */
int chfsi_abi_sizes(int64_t* system, int64_t* params, int64_t* stats);

/* ---- operator build (Section 2.3; cell-level matrices of Section 4.2) ---
 * Builds on the host, in FP64: GLL nodes and weights, the (p+1)-point Gauss
 * rule, the 1D stiffness, consistent mass and derivative matrices, the
 * reference cell matrix A_k = D_c (K^c/2 - i skew(k.G^c)/2) D_c with
 * D = M^-1/2 of the GLL-lumped overlap, the nodal potential V + |k|^2/2 and
 * the projector tables (per atom node lists and per (cell, atom) cell
 * matrices split by node multiplicity).  Then uploads them.  The operator
 * keeps a pointer to ctx, which refuses to be destroyed while the operator
 * is alive.  CHFSI_EINVAL for p outside [2, 7], a mesh of 2^29 nodes or
 * more, or a NaN or infinity anywhere in sys.  Synchronous.
 * chfsi_op_destroy() also drops a batched-filter graph the context captured
 * with this operator in it. */
int chfsi_op_build(chfsi_ctx* ctx, const chfsi_system* sys, chfsi_op** out);
int chfsi_op_destroy(chfsi_op* op);

/* The same operator with the local potential integrated per cell by the
 * (p+1)^3-point Gauss rule instead of collocated at the nodes: the
 * discrete-Hamiltonian construction of Section 4.2 (Eq. quadLocal, with all
 * cells' matrices K^loc_e[j,k] = sum_q N_j N_k V w_q |J| formed as one
 * GEMM, Eq. gemmLoc).  Every cell then has its own real cell matrix
 * D_c (K^c/2 + K^loc_e) D_c (imaginary k-part shared), stored per cell in
 * FP64 and FP32 (E x mpad^2 each: 13.7 + 6.9 GB at 24^3 cells, p = 6); the
 * diagonal keeps |k|^2/2.  All functions accept the result; the filter
 * precisions are F64 and F32 (C128 and C64 for k != 0): BF16 returns
 * CHFSI_EINVAL, as does a mesh whose packed product (mcell (mcell + 1) / 2
 * rows by E cells) reaches 2^31 entries.  Same arguments and ownership as
 * chfsi_op_build(). */
int chfsi_op_build_quadrature(chfsi_ctx* ctx, const chfsi_system* sys, chfsi_op** out);
/* M nodes, E cells, mcell = (p+1)^3 nodes per cell, nproj = 4 * natoms (0
 * without projectors), npairs = number of (cell, atom) pairs, is_complex. */
int chfsi_op_info(const chfsi_op* op, int64_t* M, int64_t* E, int32_t* mcell,
                  int32_t* nproj, int64_t* npairs, int32_t* is_complex);
/* Host copies of the built tables, for checking: node coordinates (M x 3),
 * the reference cell matrix (mcell x mcell row-major; complex operators
 * write real and imaginary parts to cell_re / cell_im, cell_im may be NULL
 * otherwise), the nodal diagonal V + |k|^2/2 (M) and D = M^-1/2 (M).  Any
 * output pointer may be NULL.  Synchronous. */
int chfsi_op_tables(const chfsi_op* op, double* xyz, double* cell_re, double* cell_im,
                    double* vdiag, double* dscale);

/* ---- H~.X (Eq. celldgemm + Algorithm 4) ---------------------------------
 * Y = H~ X for ncols columns.  X and Y are device arrays with the storage
 * type of `prec` (F64: double; F32 and BF16: float; C128: complex double;
 * C64: complex float), row-major M x ld.  X and Y must not overlap.
 * Asynchronous. */
int chfsi_apply(chfsi_op* op, const void* X, void* Y, int64_t ncols, int64_t ld, int32_t prec);

/* ---- H~.X without allocation ----------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Y = H~ X as chfsi_apply(), same arguments, layouts and kernels, but the
 * projector partials and coefficients live in a fixed file-scope device
 * scratch of 64 MiB per device (held until the process ends) instead of
 * context workspace, and the call makes no hipMalloc, hipFree or allocating
 * library call.  The scratch need is align256(nchunks * 4 * ldhp * s) +
 * natoms * 4 * ldhp * s bytes with ldhp = ncols (x2 if complex) rounded up
 * to 64 and s = 8 (F64, C128) or 4 bytes; a call that needs more returns
 * CHFSI_EINVAL before any work is enqueued (c1-size operators fit 128 FP64
 * columns).  Every call on one device shares that device's scratch, and
 * every entry a call reads it writes first, so nothing is carried over
 * between calls; calls that overlap in time on one device (different
 * streams or contexts) race.  Asynchronous. */
int chfsi_apply_noalloc(chfsi_op* op, const void* X, void* Y, int64_t ncols, int64_t ld, int32_t prec);

/* ---- upper bound of the spectrum ----------------------------------------
 * `steps`-step Lanczos run without reorthogonalisation from v0 (device, M
 * real or M complex values; NULL draws one from `seed`):
 * b_upper = theta_max(T) + ||f||, lmin_est = theta_min(T).  FP64.
 * Synchronous. */
int chfsi_bounds(chfsi_op* op, int32_t steps, const void* v0, uint64_t seed,
                 double* b_upper, double* lmin_est);

/* ---- Chebyshev filter (Eq. chebyfilter, scaled three-term recurrence) ---
 * In place on the device block X (double, or complex double for a complex
 * operator; M x ld, ncols columns): X <- T_m(Hbar) X / T_m((aL - c)/e) with
 * Hbar = (H~ - c)/e, e = (b - a)/2, c = (b + a)/2.  Requires aL < a < b.
 * `prec` is the arithmetic of the recurrence (F64/F32/BF16 real, C128/C64
 * complex); the block is converted to it and back.  Columns are processed in
 * blocks of `block` (<= 0: all at once).  Asynchronous. */
int chfsi_filter(chfsi_op* op, void* X, int64_t ncols, int64_t ld, int32_t m,
                 double a, double b, double aL, int32_t prec, int32_t block);

/* ---- Cholesky-Gram-Schmidt (Algorithm 2, RRGEP-O and Cholesky of S) ----
 * In place on the device block X (double / complex double): S = X^H X
 * (FP64, lower triangle, deterministic), S = L L^H, X <- X L^-H.
 * L_host (nullable, ncols x ncols row-major, complex interleaved for a
 * complex operator) receives L.  Returns CHFSI_ECHOL, leaving X unchanged,
 * if S is not positive definite.  Synchronous. */
int chfsi_orthonormalize(chfsi_op* op, void* X, int64_t ncols, int64_t ld, double* L_host);

/* ---- Rayleigh-Ritz (Algorithm 2, RRGEP-P, RRGEP-D, RRGEP-ST) ------------
 * X (device, orthonormal columns) is replaced by the Ritz vectors, ordered by
 * ascending Ritz value: W = H~ X, H^ = X^H W (lower triangle, mirrored),
 * H^ = Q' Theta Q'^H, X <- X Q'.  theta (host, ncols) receives the Ritz
 * values; resid (host, nullable) receives r_i = ||H~ psi_i - theta_i psi_i||.
 * FP64 throughout.  Synchronous. */
int chfsi_rayleigh_ritz(chfsi_op* op, void* X, int64_t ncols, int64_t ld, double* theta,
                        double* resid);

/* Rayleigh-Ritz through the generalised eigenproblem with spectrum splitting
 * (Algorithm 2 of Section 3.2: RRGEP-O, -P, -D, -ST-F, -ST-O), with the
 * mixed-precision scheme of Sections 3.2 and 4.4 when mixed != 0.
 * X: device, M x ld, FP64 (complex double for a complex operator), the
 * filtered block Psi_f (ncols = N columns, not orthonormal); on return it
 * holds the orthonormal basis Psi_o = Psi_f L^-H (S = Psi_f^H Psi_f = L L^H).
 * Psi_fr: device, M x ld_fr of the same type, receives the nfr highest Ritz
 * vectors Psi_f Q_fr of H^ Q = S Q D (H^ = Psi_f^H H~ Psi_f), in ascending
 * order.  theta: host, N, all generalised eigenvalues
 * ascending.  mixed: S's off-diagonal 128 x 128 blocks and H^ outside its
 * trailing nfr x nfr block are formed from FP32 copies in FP32 arithmetic
 * (FP64 between row chunks); Psi_o = FP32[Psi_f (L^-T without its diagonal)]
 * + FP64[Psi_f diag(L^-T)] (L^-H for complex data, handled through the
 * real views of the Gram and rotation kernels).  1 <= nfr <= N.  CHFSI_ECHOL if S is not positive definite.
 * Synchronous. */
int chfsi_rayleigh_ritz_split(chfsi_op* op, void* X, int64_t ncols, int64_t ld, int32_t nfr, int32_t mixed,
                              double* theta, void* Psi_fr, int64_t ld_fr);

/* ---- full solve -----------------------------------------------------------
 * X (device, double or complex double, M x ld with N + n_buf columns) holds
 * the start block on entry and the Ritz vectors on exit.  Steps: bound b;
 * CholGS + RR on X giving a = theta_{N+n_buf}, aL = theta_1; then passes of
 * (filter every block, CholGS, RR, update a and aL).  theta and resid (host,
 * N + n_buf each, resid nullable) receive the final Ritz values and residual
 * norms; stats (nullable) the timings and stats->b_upper the bound used.
 * Returns CHFSI_NOTCONV if a tolerance was requested and not met.
 * A start block that is rank deficient to working precision (repeated or
 * linearly dependent columns: its overlap matrix fails the Cholesky test)
 * is repaired once: the columns from the first dependent one on are redrawn
 * N(0, 1) from params->seed and stats->redrawn_columns says how many; a
 * second failure returns CHFSI_ECHOL.
 * Checkpoint and resume: the state between passes is X and b (a and aL are
 * recomputed from the Ritz values by the initial Rayleigh-Ritz), so a solve
 * restarted from the X it returned, with params->b_upper = stats->b_upper,
 * continues the same iteration up to rounding.  Synchronous. */
int chfsi_solve(chfsi_op* op, const chfsi_params* params, void* X, int64_t ld, double* theta,
                double* resid, chfsi_stats* stats);

/* ---- mixed-precision schedule ----------------------------------------------
 * The rule chfsi_solve() applies with params->prec_switch, for callers that
 * drive the passes themselves (chfsi_pass): given the filter precision of the
 * pass just done and max_resid[0..k] (k >= 1; entry 0 after the initial
 * Rayleigh-Ritz, entry i after pass i), returns the precision of the next
 * pass.  Host only; returns prec unchanged for k < 1 or a NULL history. */
int32_t chfsi_next_prec(int32_t prec, const double* max_resid, int32_t k, double b_upper);

/* ---- one ChFSI pass ---------------------------------------------------------
 * One pass of the loop of chfsi_solve() on the device block X (N + n_buf
 * columns, the current Ritz vectors): filter every column block of
 * params->block columns with degree params->m on [a, b] with lower end aL in
 * params->filter_prec, then CholGS and Rayleigh-Ritz in FP64.  theta and
 * resid (host, N + n_buf each; resid nullable) receive the new Ritz values
 * and residual norms.  params->nwanted, n_buf, m, block and filter_prec are
 * read; the stopping fields are ignored.  Synchronous. */
int chfsi_pass(chfsi_op* op, const chfsi_params* params, void* X, int64_t ld, double a, double b, double aL,
               double* theta, double* resid);

/* ---- Fermi level and electron density ---------------------------------------
 * Fermi-Dirac occupations f_i = 1 / (1 + exp((theta_i - mu) / kT)) of the
 * Ritz values (Section 2.1, Fermi-Dirac smearing and the electron-count
 * constraint; first step of the density-computation algorithm of Section
 * 3.2).  chfsi_fermi_level() finds mu with 2 sum_i w_i f_i = n_electrons by
 * bisection down to the spacing of doubles (the count rises monotonically
 * with mu).  theta: host, n values; weights: host, n non-negative k-point
 * weights (NULL: all 1); occ (host, n, nullable) receives f_i.  Requires
 * 0 < n_electrons < 2 sum_i w_i and kT > 0, else CHFSI_EINVAL.  Host only. */
int chfsi_fermi_level(const double* theta, int32_t n, const double* weights, double n_electrons, double kT,
                      double* mu, double* occ);

#define CHFSI_RHO_NODES 0  /* rho at the mesh nodes: M values, node order      */
#define CHFSI_RHO_GAUSS 1  /* rho at the (p+1)^3 Gauss-Legendre points of every
                              cell: E x (p+1)^3 values, cell cx + nc (cy + nc cz)
                              major, point qx + (p+1) (qy + (p+1) qz) within the
                              cell at origin + (1 + g_q) h / 2 per axis         */

/* Electron density of the density-computation algorithm of Section 3.2:
 *   rho(x) (+)= sum_c w_c |psi^_c(x)|^2,   psi^_c = M^-1/2 X_c
 * interpolated with the FE basis (nodal values at the nodes; the cell's
 * tensor-product Lagrange basis at the Gauss points).  X: device, M x ld,
 * FP64 for a real operator or complex double for a complex one (the block
 * type of chfsi_solve); w: host, ncols finite weights of any sign, e.g.
 * 2 f_i for Ritz vectors, or in the spectrum-split form 2 for an orthonormal
 * basis of the filtered space and 2 (f_i - 1) for the fractionally occupied
 * Ritz vectors, accumulated in two calls; k-point weights multiply in.
 * rho: device, overwritten (accumulate == 0) or added to.  The weights are
 * copied before the call returns (it waits for the stream once to do so);
 * the kernel itself runs asynchronously. */
int chfsi_density(chfsi_op* op, const void* X, int64_t ncols, int64_t ld, const double* w, int32_t points,
                  int32_t accumulate, double* rho);

/* ---- self-consistent field loop (Section 3, Algorithm 1) ----------------------
 * chfsi_op_set_potential: replaces the nodal local potential of a real or
 * complex operator built by chfsi_op_build() with V (device, M values, Ha);
 * |k|^2/2 is added as at build time.  chfsi_op_tables() keeps reporting the
 * build-time potential.  CHFSI_EINVAL for an operator from
 * chfsi_op_build_quadrature().  Asynchronous (synchronous when k != 0). */
int chfsi_op_set_potential(chfsi_op* op, const double* V);

/* Hartree potential of the density rho (device, M nodal values): the
 * periodic Poisson problem -lap v = 4 pi (rho - rho_bar) in the FE basis,
 * K v = 4 pi M (rho - rho_bar) with rho_bar the mean charge and
 * sum_j M_jj v_j = 0, solved as D K D u = 4 pi M^1/2 (rho - rho_bar),
 * v = D u, by Jacobi-preconditioned CG (the paper's Poisson solver) to a
 * relative residual tol, at most maxit iterations; the stiffness is applied
 * cell by cell by sum factorisation of its 1D factors.  vH: device, M values.
 * The CG scalars stay on the device and the residual is checked every 8
 * iterations, so the count is a multiple of 8 (or maxit) and the solve may
 * run up to 7 iterations past tol.  iters / relres (nullable) receive the
 * iteration count and the final relative residual.  Operators with a nodal
 * potential (real or Bloch: the problem depends on the mesh only).  Returns
 * CHFSI_NOTCONV if tol was not reached,
 * CHFSI_EDIVERGE on a non-finite residual.  Synchronous. */
int chfsi_hartree(chfsi_op* op, const double* rho, double* vH, double tol, int32_t maxit, int32_t* iters,
                  double* relres);

/* A self-consistent field loop around the eigensolver (Algorithm 1 with a
 * synthetic exchange-correlation term): per step, the Hartree potential of
 * the input density (the solve of chfsi_hartree to tol 1e-10, started from
 * the previous step's potential after the first step), V = V_ext + v_H + v_x with
 * V_ext the operator's build-time potential and LDA exchange
 * v_x = -(3 rho / pi)^(1/3), one ChFSI pass on X (four on the first step,
 * which starts by orthonormalising X; the spectrum's upper bound comes from
 * a Lanczos run on the first step and, later, from Weyl's inequality:
 * b + max_j (V_j - V_j of the first step)), the Fermi level of the nwanted lowest
 * Ritz values (kT, n_electrons), the nodal output density, and Anderson
 * mixing of the density (weight beta, the last `depth` differences,
 * M-weighted inner products).  Stops when the M-weighted norm of
 * rho_out - rho_in falls below tol or after maxit steps.
 * X: device, M x ld FP64 (complex double for a Bloch operator: one k-point,
 * its density |psi|^2 real), nwanted + n_buf columns (start block in, Ritz
 * vectors out); rho: device, M values (initial density in; the converged
 * output density, or the last mixed density if not converged, out); theta:
 * host, nwanted + n_buf Ritz values of the last step; mu_out, res_hist
 * (host, maxit values: the residual norm of every step) and iters nullable.
 * m, block: filter degree and column block as in chfsi_params.
 * rr_mode selects the Rayleigh-Ritz step of the passes after the first SCF
 * step: 0 = CholGS + Rayleigh-Ritz on all N columns and the density of the
 * Ritz vectors; 1 = Rayleigh-Ritz through the generalised problem with
 * spectrum splitting (chfsi_rayleigh_ritz_split, Algorithm 2) and the split
 * density of Algorithm 3: rho = sum over the orthonormal basis with weight
 * 2 plus the nfr highest Ritz vectors with weight 2 (f_i - 1) (buffer states
 * f_i = 0), nfr covering every state whose vacancy 1 - f_i exceeded 1e-14
 * at the previous step, plus two; 2 = the same with the mixed-precision
 * blocks of chfsi_rayleigh_ritz_split (the paper's form).  In modes 1 and 2
 * X holds the orthonormal basis (not Ritz vectors) on return.  Operators
 * with a nodal potential (V_ext is the build-time potential without
 * |k|^2 / 2); 0 < n_electrons < 2 nwanted.  On
 * return the operator holds the last step's effective potential (restore
 * the original with chfsi_op_set_potential if needed).  Returns
 * CHFSI_NOTCONV if tol was not met.  Synchronous. */
int chfsi_scf(chfsi_op* op, void* X, int64_t ld, int32_t nwanted, int32_t n_buf, int32_t m, int32_t block,
              int32_t rr_mode, double n_electrons, double kT, double beta, int32_t depth, double tol, int32_t maxit,
              double* rho, double* theta, double* mu_out, double* res_hist, int32_t* iters);

/* The same loop with k-point sampling: nk operators of one mesh (the same
 * system at nk Bloch vectors, e.g. a Monkhorst-Pack set), each with its
 * block X[k] (ld[k]; nwanted + n_buf columns, complex for k != 0) and
 * weight weights[k] (non-negative, normalised to sum 1 here; NULL: equal).
 * The density is sum_k w_k sum_i 2 f_ki |psi_ki|^2, the Fermi level is
 * taken over all k-points' nwanted lowest Ritz values with their weights
 * (n_electrons per cell: 0 < n_electrons < 2 nwanted), the Hartree
 * potential, the mixing and the stopping rule are those of chfsi_scf, and
 * the eigensolver step (passes, spectrum splitting with its own split per
 * k-point) runs for each k-point in turn.  theta: nk host arrays of
 * nwanted + n_buf values.  chfsi_scf is this call with nk = 1.  H(-k) is
 * the complex conjugate of H(k) and has the same density, so a grid closed
 * under k -> -k may be passed as one k-point of each pair with twice the
 * weight.  Synchronous. */
int chfsi_scf_kpoints(chfsi_ctx* ctx, int32_t nk, chfsi_op* const* ops, void* const* X, const int64_t* ld,
                      const double* weights, int32_t nwanted, int32_t n_buf, int32_t m, int32_t block,
                      int32_t rr_mode, double n_electrons, double kT, double beta, int32_t depth, double tol,
                      int32_t maxit, double* rho, double* const* theta, double* mu_out, double* res_hist,
                      int32_t* iters);

/* ---- batched filter (many operators, one persistent launch per step) -------
 * Applies the filter of chfsi_filter() to n independent blocks at once:
 * block q is X[q] (device, double / complex double, ncols[q] columns, ld[q])
 * of operator ops[q] with interval a[q], b[q], aL[q] (aL < a < b).  All
 * operators must share the context, the order p and the real/complex type;
 * prec is F64, F32 (real) or C128, C64 (complex).  Column blocks of `block`
 * columns (<= 0: all) of every problem are filtered together: each
 * Chebyshev step of a round is ONE launch of a persistent kernel whose work
 * list concatenates every problem's (cell, column tile) items; the per-problem
 * arguments and recurrence scalars come from device tables.  use_graph != 0
 * captures the whole sequence into a hipGraph (kept in the context and
 * replayed while the operators, buffers and shapes stay the same).  Grid
 * shape from chfsi_autotune() when tuned, else one workgroup per item.
 * Results equal chfsi_filter() on each block up to the order of the atomic
 * assembly.  Asynchronous. */
int chfsi_filter_batched(chfsi_ctx* ctx, int32_t n, chfsi_op* const* ops, void* const* X, const int64_t* ncols,
                         const int64_t* ld, int32_t m, const double* a, const double* b, const double* aL,
                         int32_t prec, int32_t block, int32_t use_graph);

/* ---- batched solve ----------------------------------------------------------
 * chfsi_solve() for n independent problems (systems and/or k-points) that
 * advance pass by pass together: the filters of all unconverged problems run
 * through chfsi_filter_batched() (with use_graph: one graph replay per pass),
 * then the CholGS and Rayleigh-Ritz steps: when every block has at most 64
 * columns, those of all active problems together (each N x N Cholesky,
 * inverse and eigensolve of all problems in one launch, two host
 * synchronisations per pass; stats t_rr then holds an even share of that
 * step), otherwise each problem's in turn.  params, X, ld,
 * theta, resid, stats are arrays of n entries (resid, stats and their entries
 * nullable); m, block and filter_prec must be equal across params and
 * prec_switch must be 0.  History arrays are filled per problem, with times
 * measured from the start of the call.  A problem stops when its own
 * criterion is met; the others continue.  Returns CHFSI_NOTCONV if any
 * tolerance was not met; a rank-deficient start block is not redrawn here
 * (CHFSI_ECHOL).  Synchronous. */
int chfsi_solve_batched(chfsi_ctx* ctx, int32_t n, chfsi_op* const* ops, const chfsi_params* params,
                        void* const* X, const int64_t* ld, double* const* theta, double* const* resid,
                        chfsi_stats* stats, int32_t use_graph);

/* ---- autotuner of the batched launch ----------------------------------------
 * Times the batched filter on a synthetic batch of four uneven boxes of order
 * p with `block` columns over launch shapes: the work item of the cell kernel
 * (a cell by 64 columns, on 4 waves, or on 2 waves where real FP32 gives each
 * wave all 64 columns; or a cell by 32 columns on half the waves) times the
 * grid (one workgroup per item, reported as grid_per_cu = 0, or a persistent
 * grid of 1..4 workgroups per CU with contiguous or strided item assignment).
 * It keeps the fastest for the key (gfx950, p, prec, block) in the context
 * and, when cache_json is not NULL, merges it into that JSON file (read
 * first, then rewritten).  Synchronous.  chfsi_load_tuning() reads such a
 * file into the context (an entry without "col_tile" takes the default
 * rule); chfsi_get_tuning() returns the shape the batched launch will use:
 * grid_per_cu, contiguous, col_tile (64 or 32; 0 = the default rule, 32 when
 * every block has at most 32 real columns, else 64) and the tuned time in ms
 * (0 when untuned); every output pointer is nullable.  Untuned single-problem
 * launches use the same default rule for their column tile. */
int chfsi_autotune(chfsi_ctx* ctx, const char* cache_json, int32_t p, int32_t prec, int32_t block);
int chfsi_load_tuning(chfsi_ctx* ctx, const char* cache_json);
int chfsi_get_tuning(chfsi_ctx* ctx, int32_t p, int32_t prec, int32_t block, int32_t* grid_per_cu,
                     int32_t* contiguous, int32_t* col_tile, double* ms);

/* ---- learned warm start -------------------------------------------------------
 * A small network maps per-node features to an initial block (an extension
 * around the paper's method; the paper starts ChFSI from the previous SCF
 * step's subspace).
 *
 * chfsi_features: F (device, float, M x 32 row-major) receives the radial
 *   features of every node: F[j][8q + k] = sum_a sum_images phi_q(a)
 *   exp(-(r - k)^2 / (2 * 0.5^2)), r = |x_j - R_a - nL| <= 10 bohr, k = 0..7,
 *   phi = (Z_a, s_a, h_s,a, h_p,a).  Asynchronous.
 * chfsi_mlp_create: network din -> hidden (tanh) -> hidden (tanh) -> dout
 *   (linear), all widths <= 128, FP32, Xavier-uniform weights drawn from
 *   `seed` (splitmix64), zero biases, Adam state zero, input normalisation
 *   mean 0 / scale 1.  The network keeps a pointer to ctx.
 * chfsi_mlp_params: flat parameter vector (host, chfsi_mlp_info nparams
 *   floats) in the order W1 (din x hidden, row-major), b1, W2, b2, W3, b3;
 *   get != 0 copies out, 0 copies in.  Synchronous.
 * chfsi_mlp_set_norm: input standardisation (F - mean) / scale (host arrays
 *   of din; scales > 0).
 * chfsi_mlp_forward: Y (device, rows x dout) = network(F (device, rows x din)).
 * chfsi_mlp_loss_grad: loss = ||Y - Q Q^T Y||^2 / ||Y||^2
 *   + 0.1 ||dout Y^T Y / ||Y||^2 - I||^2 / dout^2 for Y = network(F) and the
 *   orthonormal block Q (device, rows x nq, nq = dout); grads_host (nullable,
 *   nparams floats) receives d loss / d parameters.  Synchronous.
 * chfsi_mlp_train_step: loss_grad followed by one Adam step (lr, 0.9, 0.999,
 *   1e-8).  Synchronous (returns the loss before the step).
 * chfsi_initial_block: X (device, double, M x ld, ncols columns) receives the
 *   network's block (features of op, forward, widened to FP64; columns beyond
 *   dout drawn from `seed`), or a random N(0,1) block from `seed` when net is
 *   NULL, the operator is complex, or the network's block is non-finite or
 *   has a non-positive-definite overlap; *used_fallback says which.
 *   Synchronous. */
int chfsi_features(chfsi_op* op, float* F);
int chfsi_mlp_create(chfsi_ctx* ctx, int32_t din, int32_t hidden, int32_t dout, uint64_t seed, chfsi_mlp** out);
int chfsi_mlp_destroy(chfsi_mlp* net);
int chfsi_mlp_info(const chfsi_mlp* net, int32_t* din, int32_t* hidden, int32_t* dout, int64_t* nparams);
int chfsi_mlp_params(chfsi_mlp* net, float* host, int32_t get);
int chfsi_mlp_set_norm(chfsi_mlp* net, const float* mean, const float* scale);
int chfsi_mlp_forward(chfsi_mlp* net, const float* F, int64_t rows, float* Y);
int chfsi_mlp_loss_grad(chfsi_mlp* net, const float* F, int64_t rows, const float* Q, int32_t nq, double* loss,
                        float* grads_host);
int chfsi_mlp_train_step(chfsi_mlp* net, const float* F, int64_t rows, const float* Q, int32_t nq, float lr,
                         double* loss);
int chfsi_initial_block(chfsi_op* op, chfsi_mlp* net, uint64_t seed, void* X, int64_t ncols, int64_t ld,
                        int32_t* used_fallback);

/* ---- deterministic assembly ----------------------------------------------
 * Section 4.3 assembles the cell products Y^c into the global vector (the
 * scatter of Eq. celldgemm); the default path adds them with hardware
 * atomics, so the order in which the up to 8 cells sharing a node add into
 * it depends on workgroup timing and the result can differ from run to run
 * in the last bits.  chfsi_set_deterministic(ctx, 1) runs every H~.X of the
 * context (chfsi_apply, chfsi_apply_noalloc, the filter, the solvers, and the
 * batched filter and solve, which then run problem by problem) colour class
 * by colour class: along each axis the cells take colours 0, 1, 0, 1, ...
 * (and 2 for the last cell of an odd side), a class is a triple of axis
 * colours, no two cells of one class share a node, and the classes run in a
 * fixed order, one launch each (8 launches per H~.X for an even number of
 * cells per side, 27 for an odd one).  Results are then bitwise reproducible
 * for the same inputs, launch shapes and device.  Enabling builds the colour
 * classes of every live operator (one int32 per cell on the device); an
 * operator built later gets them at construction.  Operators with a single
 * cell per side (a cell sharing nodes with its own periodic images) cannot
 * be coloured: their H~.X calls return CHFSI_EINVAL while the mode is on.
 * The mode also covers the Hartree solve of chfsi_hartree and chfsi_scf:
 * its stiffness assembly runs by colour class as well, and the dot products
 * of its CG are summed from per-block partials in a fixed order instead of
 * by atomic adds (three more small launches per CG iteration), so a whole
 * SCF run is bitwise reproducible.  Returns CHFSI_EINVAL for a null ctx,
 * CHFSI_ENOMEM / CHFSI_EHIP if the classes cannot be uploaded (the mode then
 * stays as it was). */
int chfsi_set_deterministic(chfsi_ctx* ctx, int32_t enable);

/* ---- kernel timing ---------------------------------------------------------
 * When enabled, the library brackets every launch of the cell H~.X kernel
 * with HIP events on the context stream.  chfsi_kernel_time() waits for the
 * stream and returns the summed duration (ms), the number of launches and the
 * summed algorithmic flops of those launches since the last reset (reset != 0
 * clears the counters after reading). */
int chfsi_set_timing(chfsi_ctx* ctx, int32_t enable);
int chfsi_kernel_time(chfsi_ctx* ctx, double* total_ms, int64_t* launches, double* flops, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* CHFSI_H */
