// Context and operator internals shared by the host sources of libchfsi.
#pragma once

#include <cmath>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

using namespace chfsi;

namespace chfsi_host {

enum Slot {
  WS_R0, WS_R1, WS_R2, WS_R3,      // filter buffers
  WS_NLPART, WS_HP,                // projector partials / scaled coefficients
  WS_GPART, WS_G, WS_S, WS_Z, WS_Z2,
  WS_W, WS_X2, WS_HPSI,            // M x N work blocks
  WS_RPART, WS_VEC, WS_SMALL, WS_EIG, WS_INFO,
  WS_BATCH, WS_BTAB,               // batched filter buffers and descriptor tables
  WS_DENS,                         // density weights
  WS_RR_G, WS_RR_S, WS_RR_H, WS_RR_Z, // split Rayleigh-Ritz: lower Gram, S, H^, rotation
  WS_X32, WS_W32, WS_C32,          // FP32 copies of X, H X and the FP32 rotation
  WS_SCF,                          // SCF vectors (potentials, densities, CG, mixing history)
  WS_CG,                           // CG scalars and the residual history of one check interval
  WS_PFR,                          // SCF: the highest Ritz vectors of the split Rayleigh-Ritz
  WS_SUBB,                         // batched small subspace step: per-problem blocks and matrices
  WS_COUNT
};

}  // namespace chfsi_host

using namespace chfsi_host;

struct chfsi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  rocblas_handle blas = nullptr;
  std::string err;
  void* ws[WS_COUNT] = {};
  size_t ws_size[WS_COUNT] = {};
  // opt-in timing of the cell kernel: event pairs not yet read, totals
  bool timing = false;
  // deterministic assembly (chfsi_set_deterministic): every H~.X launch runs
  // colour class by colour class
  bool deterministic = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<double> pending_flops;
  double t_ms = 0.0, t_flops = 0.0;
  int64_t t_launches = 0;
  // batched launches: tuned persistent-grid shapes per (arch, p, prec, block)
  // col_tile: columns per work item of the cell kernel (64 or 32; 0: 32 for
  // blocks of at most 32 real columns, else 64)
  struct Tuning { int grid_per_cu = 2; int contiguous = 1; int col_tile = 0; double ms = 0.0; };
  std::map<std::string, Tuning> tuning;
  int ncu = 0;
  void* pinned = nullptr;           // host staging of descriptor tables
  size_t pinned_size = 0;
  hipStream_t cap_stream = nullptr; // private stream that graphs are captured on
  hipGraph_t graph = nullptr;       // captured batched filter
  hipGraphExec_t gexec = nullptr;
  std::string gkey;
  // live operators and networks: the context refuses to be destroyed while
  // any is alive (they hold its stream and scratch), and a captured graph is
  // keyed by operator ids, which are never reused, instead of addresses
  std::set<const void*> live_ops, live_mlps;
  // device address of this device's fixed scratch (chfsi_apply_noalloc),
  // resolved once at context creation, or null with the reason
  void* scratch = nullptr;
  std::string scratch_err;
  uint64_t next_op_id = 1;
};

struct chfsi_op {
  chfsi_ctx* ctx = nullptr;
  uint64_t id = 0;                   // unique within the context
  HostTables t;                      // host copies (large projector arrays dropped)
  int64_t npairs = 0;
  // device tables
  void* A64 = nullptr;  void* Ai64 = nullptr;   // swizzled cell matrix, double
  void* A32 = nullptr;  void* Ai32 = nullptr;   // float
  void* Abf = nullptr;                          // bf16, 16x16x32 operand order
  double* vdiag = nullptr;
  double* dscale = nullptr;     // M^-1/2 per node (density)
  int64_t astride = 0;          // per-cell real cell matrices (quadrature potential): elements per cell
  double* scf_tab = nullptr;    // SCF tables, 5 x M: V_ext, M^1/2, M, diag(D K D), zeros
  int64_t* atom_ptr = nullptr;
  int32_t* atom_node = nullptr;
  double* atom_val = nullptr;
  int32_t* chunk_atom = nullptr;
  int64_t* chunk_begin = nullptr;
  int32_t* atom_chunk_ptr = nullptr;
  int nchunks = 0;
  double* hcoef = nullptr;
  int32_t* pair_ptr = nullptr;
  int32_t* pair_atom = nullptr;
  void* pair_re64 = nullptr; void* pair_im64 = nullptr;
  void* pair_re32 = nullptr; void* pair_im32 = nullptr;
  double* d_x1d = nullptr;      // node coordinates along one axis (features)
  double* d_atoms = nullptr;    // atom table (features)
  // colour classes of the cells for deterministic assembly: the cells of
  // class k are colour_cells[colour_off[k] .. colour_off[k + 1]) (device);
  // built when deterministic assembly is first switched on for the operator
  int32_t* colour_cells = nullptr;
  std::vector<int> colour_off;
  std::vector<void*> allocs;
};

namespace chfsi_host {

extern thread_local std::string g_create_err;

inline int fail(chfsi_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ctx, CHFSI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define RB_TRY(ctx, expr)                                                                 \
  do {                                                                                    \
    rocblas_status s_ = (expr);                                                           \
    if (s_ != rocblas_status_success)                                                     \
      return fail(ctx, CHFSI_EHIP, std::string(#expr) + ": rocblas status " +             \
                                       std::to_string(static_cast<int>(s_)));             \
  } while (0)

#define CHECK(expr)            \
  do {                         \
    int r_ = (expr);           \
    if (r_ < 0) return r_;     \
  } while (0)

// Grow-only scratch slot.
inline int ws_get(chfsi_ctx* c, int slot, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  if (c->ws_size[slot] < bytes) {
    if (c->ws[slot]) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      HIP_TRY(c, hipFree(c->ws[slot]));
      c->ws[slot] = nullptr;
      c->ws_size[slot] = 0;
    }
    const size_t b = (bytes + 4095) / 4096 * 4096;
    hipError_t e = hipMalloc(&c->ws[slot], b);
    if (e != hipSuccess) {
      c->ws[slot] = nullptr;
      return fail(c, CHFSI_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
    c->ws_size[slot] = b;
  }
  *out = c->ws[slot];
  return 0;
}

// splitmix64 (Steele, Lea, Flood 2014) + Box-Muller: the library's own
// generator for start vectors when the caller gives none.
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  }
};

}  // namespace chfsi_host
