// Learned warm start for ChFSI: a small network maps per-node radial features
// of the atoms to an initial block, replacing the random start block of the
// first Rayleigh-Ritz step.  Training and inference run in the FP32 kernels of
// kernels_mlp.hip; the library falls back to a random block whenever the
// network's block is non-finite or its overlap matrix is not positive
// definite.
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "context.h"

using namespace chfsi;

namespace {

constexpr double kEta = 0.5;   // radial width (bohr)
constexpr double kRcut = 10.0; // feature cutoff (bohr)
constexpr int kDin = 32;

enum MlpSlot { M_F, M_FN, M_A1, M_A2, M_Y, M_DY, M_T1, M_T2, M_GPART, M_CPART, M_DPART, M_SMALL, M_G, M_D, M_P,
               M_X2, M_COUNT };

}  // namespace

struct chfsi_mlp {
  chfsi_ctx* ctx = nullptr;
  int din = 0, hid = 0, dout = 0;
  int64_t np = 0;
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  float* params = nullptr;
  float* grads = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* mean = nullptr;
  float* stdv = nullptr;
  int t = 0;
  void* ws[M_COUNT] = {};
  size_t wss[M_COUNT] = {};
};

namespace {

int mws(chfsi_mlp* n, int slot, size_t bytes, void** out) {
  chfsi_ctx* c = n->ctx;
  if (bytes == 0) bytes = 256;
  if (n->wss[slot] < bytes) {
    if (n->ws[slot]) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      HIP_TRY(c, hipFree(n->ws[slot]));
      n->ws[slot] = nullptr;
      n->wss[slot] = 0;
    }
    const size_t b = (bytes + 4095) / 4096 * 4096;
    if (hipMalloc(&n->ws[slot], b) != hipSuccess) {
      n->ws[slot] = nullptr;
      return fail(c, CHFSI_ENOMEM, "hipMalloc of network workspace failed");
    }
    n->wss[slot] = b;
  }
  *out = n->ws[slot];
  return 0;
}

float* fws(chfsi_mlp* n, int slot, int64_t count, int* rc) {
  void* p = nullptr;
  *rc = mws(n, slot, static_cast<size_t>(count) * 4, &p);
  return static_cast<float*>(p);
}

int dot_sum(chfsi_mlp* n, const float* x, const float* y, int64_t len, double* out) {
  chfsi_ctx* c = n->ctx;
  void* part;
  CHECK(mws(n, M_DPART, static_cast<size_t>(mlp_dot_blocks()) * 8, &part));
  HIP_TRY(c, mlp_dot(x, y, len, static_cast<double*>(part), c->stream));
  std::vector<double> h(mlp_dot_blocks());
  HIP_TRY(c, hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (double v : h) s += v;
  *out = s;
  return 0;
}

// forward pass on n rows of raw features F; Y (n x dout) may be external
int forward(chfsi_mlp* net, const float* F, int64_t n, float* Yext) {
  chfsi_ctx* c = net->ctx;
  int rc = 0;
  float* Fn = fws(net, M_FN, n * net->din, &rc); CHECK(rc);
  float* A1 = fws(net, M_A1, n * net->hid, &rc); CHECK(rc);
  float* A2 = fws(net, M_A2, n * net->hid, &rc); CHECK(rc);
  float* Y = Yext;
  if (!Y) { Y = fws(net, M_Y, n * net->dout, &rc); CHECK(rc); }
  const float* P = net->params;
  HIP_TRY(c, mlp_normalize(F, net->mean, net->stdv, Fn, n, net->din, c->stream));
  HIP_TRY(c, mlp_gemm(Fn, net->din, P + net->oW1, net->hid, 1, A1, net->hid, n, net->din, net->hid, 1,
                      P + net->ob1, nullptr, 0, c->stream));
  HIP_TRY(c, mlp_gemm(A1, net->hid, P + net->oW2, net->hid, 1, A2, net->hid, n, net->hid, net->hid, 1,
                      P + net->ob2, nullptr, 0, c->stream));
  HIP_TRY(c, mlp_gemm(A2, net->hid, P + net->oW3, net->dout, 1, Y, net->dout, n, net->hid, net->dout, 0,
                      P + net->ob3, nullptr, 0, c->stream));
  return 0;
}

// X = (G + eps I)^-1 P^T (D x nq) for the symmetric G (D x D, float,
// row-major) and P (nq x D), by Cholesky in FP64; captured = tr(P X).
// False if G + eps I is not positive definite.
bool coverage_solve(const std::vector<float>& Gf, const std::vector<float>& Pf, int D, int nq, double eps,
                    std::vector<double>& X, double* captured) {
  std::vector<double> L(static_cast<size_t>(D) * D, 0.0);
  const double ridge = eps;
  for (int i = 0; i < D; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = 0.5 * (static_cast<double>(Gf[static_cast<size_t>(i) * D + j]) + Gf[static_cast<size_t>(j) * D + i]);
      if (i == j) v += ridge;
      for (int k = 0; k < j; ++k) v -= L[static_cast<size_t>(i) * D + k] * L[static_cast<size_t>(j) * D + k];
      if (i == j) {
        if (!(v > 0.0)) return false;
        L[static_cast<size_t>(i) * D + i] = std::sqrt(v);
      } else {
        L[static_cast<size_t>(i) * D + j] = v / L[static_cast<size_t>(j) * D + j];
      }
    }
  X.assign(static_cast<size_t>(D) * nq, 0.0);
  for (int q = 0; q < nq; ++q) {
    // L y = P^T[:, q], then L^T x = y
    std::vector<double> y(D);
    for (int i = 0; i < D; ++i) {
      double v = Pf[static_cast<size_t>(q) * D + i];
      for (int k = 0; k < i; ++k) v -= L[static_cast<size_t>(i) * D + k] * y[k];
      y[i] = v / L[static_cast<size_t>(i) * D + i];
    }
    for (int i = D - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < D; ++k) v -= L[static_cast<size_t>(k) * D + i] * X[static_cast<size_t>(k) * nq + q];
      X[static_cast<size_t>(i) * nq + q] = v / L[static_cast<size_t>(i) * D + i];
    }
  }
  double t = 0.0;
  for (int q = 0; q < nq; ++q)
    for (int i = 0; i < D; ++i) t += static_cast<double>(Pf[static_cast<size_t>(q) * D + i]) * X[static_cast<size_t>(i) * nq + q];
  *captured = t;
  return true;
}

// subspace loss of the network output against Q (n x nq, ldq, orthonormal);
// with grads, the gradient of the loss w.r.t. every parameter is written to
// net->grads.
int loss_grad(chfsi_mlp* net, const float* F, int64_t n, const float* Q, int64_t ldq, int nq, double* loss,
              bool grads) {
  chfsi_ctx* c = net->ctx;
  int rc = 0;
  const int H = net->hid, D = net->dout;
  CHECK(forward(net, F, n, nullptr));
  float* Y = static_cast<float*>(net->ws[M_Y]);
  float* A1 = static_cast<float*>(net->ws[M_A1]);
  float* A2 = static_cast<float*>(net->ws[M_A2]);
  float* Fn = static_cast<float*>(net->ws[M_FN]);
  float* T1 = fws(net, M_T1, n * std::max(H, D), &rc); CHECK(rc);
  float* T2 = fws(net, M_T2, n * std::max(H, D), &rc); CHECK(rc);
  float* dY = fws(net, M_DY, n * D, &rc); CHECK(rc);
  float* gpart = fws(net, M_GPART, static_cast<int64_t>(mlp_gram_partial_bytes(n) / 4), &rc); CHECK(rc);
  float* Pm = fws(net, M_P, static_cast<int64_t>(nq) * D, &rc); CHECK(rc);
  float* G = fws(net, M_G, static_cast<int64_t>(D) * D, &rc); CHECK(rc);
  float* Dm = fws(net, M_D, static_cast<int64_t>(D) * D, &rc); CHECK(rc);
  void* small;
  CHECK(mws(net, M_SMALL, 64, &small));
  // P = Q^T Y ; R = Y - Q P (in T1)
  HIP_TRY(c, mlp_gram(Q, ldq, nq, Y, D, D, n, gpart, Pm, D, c->stream));
  HIP_TRY(c, mlp_gemm(Q, ldq, Pm, D, 1, T1, D, n, nq, D, 2, nullptr, Y, D, c->stream));
  double s, r2;
  CHECK(dot_sum(net, Y, Y, n * D, &s));
  CHECK(dot_sum(net, T1, T1, n * D, &r2));
  if (!(s > 0.0) || !std::isfinite(s)) return fail(c, CHFSI_EDIVERGE, "network output is zero or non-finite");
  // G = Y^T Y ; D = (D/s) G - I ; inner = sum D.G ; sumD2 = sum D.D
  HIP_TRY(c, mlp_gram(Y, D, D, Y, D, D, n, gpart, G, D, c->stream));
  HIP_TRY(c, mlp_loss_small(G, D, s, Dm, static_cast<double*>(small), c->stream));
  double hs[2];
  HIP_TRY(c, hipMemcpyAsync(hs, small, 16, hipMemcpyDeviceToHost, c->stream));
  // coverage term mu (1 - tr(P G^-1 P^T) / nq) (P = Q^T Y, G = Y^T Y): the
  // D x D algebra runs on the host in FP64
  std::vector<float> hP(static_cast<size_t>(nq) * D), hG(static_cast<size_t>(D) * D), hDm(static_cast<size_t>(D) * D);
  HIP_TRY(c, hipMemcpyAsync(hP.data(), Pm, hP.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(hG.data(), G, hG.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(hDm.data(), Dm, hDm.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  // ridge eps = delta s / D (delta = 1 % of the mean eigenvalue of G)
  const double lam = 0.1, nn = D, mu = 1.0, delta = 0.01;
  std::vector<double> Xc;   // (G + eps I)^-1 P^T (D x nq, row-major)
  double captured = 0.0;
  if (!coverage_solve(hG, hP, D, nq, delta * s / nn, Xc, &captured))
    return fail(c, CHFSI_EDIVERGE, "network output overlap is not positive definite");
  *loss = r2 / s + lam * hs[1] / (nn * nn) + mu * (1.0 - captured / nq);
  if (!grads) return 0;
  double xx = 0.0;
  for (double v : Xc) xx += v * v;
  // dY = (2/s) R + (-2 r2/s^2 - (lam/n^2)(4n/s^2) inner) Y + (lam/n^2)(4n/s) Y D
  //      + (mu / nq) (-2 Q X^T + 2 Y X X^T + (2 delta / n) ||X||^2 Y);
  // the coverage part is folded into the two products: P -> P + k1 X^T in
  // R = Y - Q P and D -> D + k2 X X^T in Y D, and into the Y coefficient
  const double c1 = 2.0 / s;
  const double c2 = -2.0 * r2 / (s * s) - (lam / (nn * nn)) * (4.0 * nn / (s * s)) * hs[0] +
                    (mu / nq) * (2.0 * delta / nn) * xx;
  const double c3 = (lam / (nn * nn)) * (4.0 * nn / s);
  const double k1 = (2.0 * mu / nq) / c1, k2 = (2.0 * mu / nq) / c3;
  for (int i = 0; i < nq; ++i)
    for (int j = 0; j < D; ++j)
      hP[static_cast<size_t>(i) * D + j] += static_cast<float>(k1 * Xc[static_cast<size_t>(j) * nq + i]);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      double acc = 0.0;
      for (int q = 0; q < nq; ++q) acc += Xc[static_cast<size_t>(i) * nq + q] * Xc[static_cast<size_t>(j) * nq + q];
      hDm[static_cast<size_t>(i) * D + j] += static_cast<float>(k2 * acc);
    }
  HIP_TRY(c, hipMemcpyAsync(Pm, hP.data(), hP.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(Dm, hDm.data(), hDm.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, mlp_gemm(Q, ldq, Pm, D, 1, T1, D, n, nq, D, 2, nullptr, Y, D, c->stream));
  HIP_TRY(c, mlp_gemm(Y, D, Dm, D, 1, T2, D, n, D, D, 0, nullptr, nullptr, 0, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));   // the host copies above are reused on return
  HIP_TRY(c, mlp_combine(static_cast<float>(c1), T1, static_cast<float>(c2), Y, static_cast<float>(c3), T2, dY,
                         n * D, c->stream));
  // backward through the three layers
  void* cpart;
  CHECK(mws(net, M_CPART, mlp_colsum_partial_bytes(n, std::max(H, D)), &cpart));
  float* g = net->grads;
  const float* P = net->params;
  HIP_TRY(c, mlp_gram(A2, H, H, dY, D, D, n, gpart, g + net->oW3, D, c->stream));
  HIP_TRY(c, mlp_colsum(dY, D, D, n, static_cast<double*>(cpart), g + net->ob3, c->stream));
  HIP_TRY(c, mlp_gemm(dY, D, P + net->oW3, 1, D, T1, H, n, D, H, 3, nullptr, A2, H, c->stream));   // dZ2
  HIP_TRY(c, mlp_gram(A1, H, H, T1, H, H, n, gpart, g + net->oW2, H, c->stream));
  HIP_TRY(c, mlp_colsum(T1, H, H, n, static_cast<double*>(cpart), g + net->ob2, c->stream));
  HIP_TRY(c, mlp_gemm(T1, H, P + net->oW2, 1, H, T2, H, n, H, H, 3, nullptr, A1, H, c->stream));   // dZ1
  HIP_TRY(c, mlp_gram(Fn, net->din, net->din, T2, H, H, n, gpart, g + net->oW1, H, c->stream));
  HIP_TRY(c, mlp_colsum(T2, H, H, n, static_cast<double*>(cpart), g + net->ob1, c->stream));
  return 0;
}

int ensure_feature_tables(chfsi_op* op) {
  chfsi_ctx* c = op->ctx;
  if (!op->d_x1d) {
    void* p;
    HIP_TRY(c, hipMalloc(&p, op->t.x1d.size() * 8));
    op->allocs.push_back(p);
    HIP_TRY(c, hipMemcpy(p, op->t.x1d.data(), op->t.x1d.size() * 8, hipMemcpyHostToDevice));
    op->d_x1d = static_cast<double*>(p);
  }
  if (!op->d_atoms && op->t.natoms > 0) {
    void* p;
    HIP_TRY(c, hipMalloc(&p, op->t.atoms.size() * 8));
    op->allocs.push_back(p);
    HIP_TRY(c, hipMemcpy(p, op->t.atoms.data(), op->t.atoms.size() * 8, hipMemcpyHostToDevice));
    op->d_atoms = static_cast<double*>(p);
  }
  return 0;
}

int features(chfsi_op* op, float* F) {
  chfsi_ctx* c = op->ctx;
  CHECK(ensure_feature_tables(op));
  if (op->t.natoms == 0) {
    HIP_TRY(c, hipMemsetAsync(F, 0, static_cast<size_t>(op->t.M) * kDin * 4, c->stream));
    return 0;
  }
  const int kimg = static_cast<int>(std::ceil(kRcut / op->t.L)) + 1;
  HIP_TRY(c, launch_features(op->d_x1d, op->t.n, op->t.L, op->d_atoms, op->t.natoms, kimg, kEta, kRcut, F,
                             c->stream));
  return 0;
}

}  // namespace

extern "C" {

int chfsi_features(chfsi_op* op, float* F) {
  if (!op) return CHFSI_EINVAL;
  if (!F) return fail(op->ctx, CHFSI_EINVAL, "null output");
  return features(op, F);
}

int chfsi_mlp_create(chfsi_ctx* ctx, int32_t din, int32_t hidden, int32_t dout, uint64_t seed, chfsi_mlp** out) {
  if (!ctx) return CHFSI_EINVAL;
  if (!out) return fail(ctx, CHFSI_EINVAL, "null output");
  *out = nullptr;
  if (din < 1 || din > 128 || hidden < 1 || hidden > 128 || dout < 1 || dout > 128)
    return fail(ctx, CHFSI_EINVAL, "network widths must be in [1, 128]");
  std::unique_ptr<chfsi_mlp> n(new chfsi_mlp());
  n->ctx = ctx;
  n->din = din;
  n->hid = hidden;
  n->dout = dout;
  n->oW1 = 0;
  n->ob1 = n->oW1 + static_cast<int64_t>(din) * hidden;
  n->oW2 = n->ob1 + hidden;
  n->ob2 = n->oW2 + static_cast<int64_t>(hidden) * hidden;
  n->oW3 = n->ob2 + hidden;
  n->ob3 = n->oW3 + static_cast<int64_t>(hidden) * dout;
  n->np = n->ob3 + dout;
  // Xavier-uniform weights (splitmix64 stream), zero biases
  std::vector<float> h(n->np, 0.f);
  SplitMix g{seed};
  auto xavier = [&](int64_t off, int fi, int fo) {
    const double lim = std::sqrt(6.0 / (fi + fo));
    for (int64_t i = 0; i < static_cast<int64_t>(fi) * fo; ++i) h[off + i] = static_cast<float>((2.0 * g.uniform() - 1.0) * lim);
  };
  xavier(n->oW1, din, hidden);
  xavier(n->oW2, hidden, hidden);
  xavier(n->oW3, hidden, dout);
  std::vector<float> zero(n->np, 0.f), ones(din, 1.f), zin(din, 0.f);
  float** bufs[6] = {&n->params, &n->grads, &n->m, &n->v, &n->mean, &n->stdv};
  const int64_t sizes[6] = {n->np, n->np, n->np, n->np, din, din};
  const float* init[6] = {h.data(), zero.data(), zero.data(), zero.data(), zin.data(), ones.data()};
  for (int i = 0; i < 6; ++i) {
    void* p = nullptr;
    if (hipMalloc(&p, sizes[i] * 4) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipFree(*bufs[j]);
      return fail(ctx, CHFSI_ENOMEM, "network allocation failed");
    }
    *bufs[i] = static_cast<float*>(p);
    HIP_TRY(ctx, hipMemcpy(p, init[i], sizes[i] * 4, hipMemcpyHostToDevice));
  }
  ctx->live_mlps.insert(n.get());
  *out = n.release();
  return 0;
}

int chfsi_mlp_destroy(chfsi_mlp* n) {
  if (!n) return 0;
  (void)hipStreamSynchronize(n->ctx->stream);
  n->ctx->live_mlps.erase(n);
  float* bufs[6] = {n->params, n->grads, n->m, n->v, n->mean, n->stdv};
  for (float* b : bufs) if (b) (void)hipFree(b);
  for (int i = 0; i < M_COUNT; ++i) if (n->ws[i]) (void)hipFree(n->ws[i]);
  delete n;
  return 0;
}

int chfsi_mlp_info(const chfsi_mlp* n, int32_t* din, int32_t* hidden, int32_t* dout, int64_t* nparams) {
  if (!n) return CHFSI_EINVAL;
  if (din) *din = n->din;
  if (hidden) *hidden = n->hid;
  if (dout) *dout = n->dout;
  if (nparams) *nparams = n->np;
  return 0;
}

int chfsi_mlp_params(chfsi_mlp* n, float* host, int32_t get) {
  if (!n || !host) return CHFSI_EINVAL;
  chfsi_ctx* c = n->ctx;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (get) HIP_TRY(c, hipMemcpy(host, n->params, n->np * 4, hipMemcpyDeviceToHost));
  else HIP_TRY(c, hipMemcpy(n->params, host, n->np * 4, hipMemcpyHostToDevice));
  return 0;
}

int chfsi_mlp_set_norm(chfsi_mlp* n, const float* mean, const float* stdv) {
  if (!n || !mean || !stdv) return CHFSI_EINVAL;
  for (int i = 0; i < n->din; ++i)
    if (!(stdv[i] > 0.f)) return fail(n->ctx, CHFSI_EINVAL, "feature scales must be positive");
  HIP_TRY(n->ctx, hipMemcpy(n->mean, mean, n->din * 4, hipMemcpyHostToDevice));
  HIP_TRY(n->ctx, hipMemcpy(n->stdv, stdv, n->din * 4, hipMemcpyHostToDevice));
  return 0;
}

int chfsi_mlp_forward(chfsi_mlp* n, const float* F, int64_t rows, float* Y) {
  if (!n) return CHFSI_EINVAL;
  if (!F || !Y || rows < 1) return fail(n->ctx, CHFSI_EINVAL, "bad arguments");
  return forward(n, F, rows, Y);
}

int chfsi_mlp_loss_grad(chfsi_mlp* n, const float* F, int64_t rows, const float* Q, int32_t nq, double* loss,
                        float* grads_host) {
  if (!n) return CHFSI_EINVAL;
  if (!F || !Q || !loss || rows < 1 || nq < 1 || nq > 128) return fail(n->ctx, CHFSI_EINVAL, "bad arguments");
  CHECK(loss_grad(n, F, rows, Q, nq, nq, loss, grads_host != nullptr));
  if (grads_host) {
    HIP_TRY(n->ctx, hipMemcpyAsync(grads_host, n->grads, n->np * 4, hipMemcpyDeviceToHost, n->ctx->stream));
    HIP_TRY(n->ctx, hipStreamSynchronize(n->ctx->stream));
  }
  return 0;
}

int chfsi_mlp_train_step(chfsi_mlp* n, const float* F, int64_t rows, const float* Q, int32_t nq, float lr,
                         double* loss) {
  if (!n) return CHFSI_EINVAL;
  if (!F || !Q || !loss || rows < 1 || nq < 1 || nq > 128 || !(lr > 0.f))
    return fail(n->ctx, CHFSI_EINVAL, "bad arguments");
  CHECK(loss_grad(n, F, rows, Q, nq, nq, loss, true));
  n->t += 1;
  HIP_TRY(n->ctx, mlp_adam(n->params, n->grads, n->m, n->v, n->np, lr, 0.9f, 0.999f, 1e-8f, n->t, n->ctx->stream));
  return 0;
}

int chfsi_initial_block(chfsi_op* op, chfsi_mlp* net, uint64_t seed, void* Xv, int64_t ncols, int64_t ld,
                        int32_t* used_fallback) {
  if (!op) return CHFSI_EINVAL;
  chfsi_ctx* c = op->ctx;
  if (!Xv || ncols < 1 || ld < ncols || ncols > op->t.M) return fail(c, CHFSI_EINVAL, "bad block");
  const int cf = op->t.cplx ? 2 : 1;
  const int64_t M = op->t.M;
  double* X = static_cast<double*>(Xv);
  bool ok = false;
  if (net && !op->t.cplx && net->din == kDin) {
    int rc = 0;
    float* F = fws(net, M_F, M * kDin, &rc); CHECK(rc);
    float* Y = fws(net, M_Y, M * net->dout, &rc); CHECK(rc);
    CHECK(features(op, F));
    CHECK(forward(net, F, M, Y));
    double s = 0.0;
    CHECK(dot_sum(net, Y, Y, M * net->dout, &s));
    const int64_t nn = std::min<int64_t>(ncols, net->dout);
    if (std::isfinite(s) && s > 0.0) {
      HIP_TRY(c, launch_convert(X, ld, CHFSI_F64, Y, net->dout, CHFSI_F32, M, nn, c->stream));
      if (ncols > nn) {
        std::vector<double> h(static_cast<size_t>(M) * (ncols - nn));
        SplitMix g{seed};
        for (auto& x : h) x = g.normal();
        void* tmp;
        CHECK(mws(net, M_X2, h.size() * 8, &tmp));
        HIP_TRY(c, hipMemcpy(tmp, h.data(), h.size() * 8, hipMemcpyHostToDevice));
        HIP_TRY(c, launch_convert(X + nn, ld, CHFSI_F64, tmp, ncols - nn, CHFSI_F64, M, ncols - nn, c->stream));
      }
      // overlap matrix must be positive definite (Cholesky of X^T X)
      const int nc = static_cast<int>(ncols);
      void *part, *G, *S, *info;
      CHECK(ws_get(c, WS_GPART, gram_partial_bytes(M, nc, ld), &part));
      CHECK(ws_get(c, WS_G, static_cast<size_t>(nc) * nc * 8, &G));
      CHECK(ws_get(c, WS_S, static_cast<size_t>(nc) * nc * 8, &S));
      CHECK(ws_get(c, WS_INFO, 64, &info));
      HIP_TRY(c, launch_gram(X, ld, X, ld, M, nc, static_cast<double*>(part), static_cast<double*>(G), nc, c->stream));
      HIP_TRY(c, launch_sym_from_lower(static_cast<double*>(G), nc, static_cast<double*>(S), nc, c->stream));
      RB_TRY(c, rocsolver_dpotrf(c->blas, rocblas_fill_lower, nc, static_cast<double*>(S), nc,
                                 static_cast<rocblas_int*>(info)));
      rocblas_int hinfo = 1;
      HIP_TRY(c, hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      ok = (hinfo == 0);
    }
  }
  if (used_fallback) *used_fallback = ok ? 0 : 1;
  if (!ok) {
    std::vector<double> h(static_cast<size_t>(M) * ncols * cf);
    SplitMix g{seed};
    for (auto& x : h) x = g.normal();
    HIP_TRY(c, hipMemcpy2D(X, ld * cf * 8, h.data(), ncols * cf * 8, ncols * cf * 8, M, hipMemcpyHostToDevice));
  }
  return 0;
}

}  // extern "C"
