// Host construction of the spectral finite-element operator tables
// (DFT-FE 1.0, Section 2.3: FE expansion on GLL nodes, discrete H^loc and
// H^nl, GLL-lumped overlap and the Loewdin transform; Section 4.2: cell-level
// matrices; Section 4.3 and Algorithm 4: cell-level projector matrices).
//
// Everything here is FP64 and runs once per operator; the kernels only read
// the resulting tables.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <unordered_map>

#include "internal.h"

namespace chfsi {
namespace {

// Legendre polynomial P_n(x) and its derivative from the three-term recurrence
// (n + 1) P_{n+1} = (2n + 1) x P_n - n P_{n-1}; valid for |x| < 1 for dP.
void legendre_pd(int n, double x, double& P, double& dP) {
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  double p0 = 1.0, p1 = x;
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

// Gauss-Lobatto-Legendre nodes (end points and roots of P_p') and weights
// 2 / (p (p + 1) P_p(x)^2).  Newton iteration on P_p' with the Legendre
// equation giving P_p'' = (2 x P_p' - p (p + 1) P_p) / (1 - x^2).
void gll_rule(int p, std::vector<double>& x, std::vector<double>& w) {
  x.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre_pd(p, t, P, dP);
      const double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
      const double dt = dP / d2P;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = t;
  }
  std::sort(x.begin(), x.end());
  for (int i = 0; i <= p; ++i) {
    double P, dP;
    if (i == 0 || i == p) {
      P = (i == p || p % 2 == 0) ? 1.0 : -1.0;  // P_p(+-1) = (+-1)^p
    } else {
      legendre_pd(p, x[i], P, dP);
    }
    w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
}

// n-point Gauss-Legendre rule: roots of P_n, weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double P = 0, dP = 1;
    for (int it = 0; it < 100; ++it) {
      legendre_pd(n, t, P, dP);
      const double dt = P / dP;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    legendre_pd(n, t, P, dP);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
  }
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(n), ws(n);
  for (int i = 0; i < n; ++i) { xs[i] = x[ord[i]]; ws[i] = w[ord[i]]; }
  x.swap(xs);
  w.swap(ws);
}

// Lagrange basis l_a on `nodes` and its derivative, at point t.
void lagrange_at(const std::vector<double>& nodes, double t, std::vector<double>& l,
                 std::vector<double>& dl) {
  const int n = static_cast<int>(nodes.size());
  l.assign(n, 0.0);
  dl.assign(n, 0.0);
  for (int a = 0; a < n; ++a) {
    double den = 1.0, num = 1.0;
    for (int b = 0; b < n; ++b)
      if (b != a) { den *= nodes[a] - nodes[b]; num *= t - nodes[b]; }
    l[a] = num / den;
    double s = 0.0;
    for (int c = 0; c < n; ++c) {
      if (c == a) continue;
      double prod = 1.0;
      for (int b = 0; b < n; ++b)
        if (b != a && b != c) prod *= t - nodes[b];
      s += prod;
    }
    dl[a] = s / den;
  }
}

}  // namespace

void swizzle_cell_matrix(const double* A, int mcell, int mpad, double* out) {
  const int rts = mpad / 16, kss = mpad / 4;
  for (int rt = 0; rt < rts; ++rt)
    for (int ks = 0; ks < kss; ++ks)
      for (int lane = 0; lane < 64; ++lane) {
        const int r = rt * 16 + lane % 16, k = ks * 4 + lane / 16;
        out[(static_cast<size_t>(rt) * kss + ks) * 64 + lane] =
            (r < mcell && k < mcell) ? A[static_cast<size_t>(r) * mcell + k] : 0.0;
      }
}

int mpad32_of(int p) { return (mcell_of(p) + 31) / 32 * 32; }

uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<uint16_t>(u >> 16);
}

void swizzle_cell_matrix_bf16(const double* A, int mcell, uint16_t* out) {
  int p = 1;
  while (mcell_of(p) < mcell) ++p;
  const int mp = mpad32_of(p);
  const int rts = mp / 16, kss = mp / 32;
  for (int rt = 0; rt < rts; ++rt)
    for (int ks = 0; ks < kss; ++ks)
      for (int lane = 0; lane < 64; ++lane)
        for (int j = 0; j < 8; ++j) {
          const int r = rt * 16 + lane % 16, k = ks * 32 + 8 * (lane / 16) + j;
          const float v = (r < mcell && k < mcell) ? static_cast<float>(A[static_cast<size_t>(r) * mcell + k]) : 0.f;
          out[((static_cast<size_t>(rt) * kss + ks) * 64 + lane) * 8 + j] = bf16_rne(v);
        }
}

void gauss_legendre_rule(int n, std::vector<double>& x, std::vector<double>& w) { gauss_rule(n, x, w); }

std::string build_tables(const chfsi_system& sys, HostTables& t) {
  const int p = sys.p, nc = sys.ncell, q = p + 1;
  t.p = p;
  t.ncell = nc;
  t.n = nc * p;
  t.M = static_cast<int64_t>(t.n) * t.n * t.n;
  t.E = static_cast<int64_t>(nc) * nc * nc;
  t.mcell = q * q * q;
  t.mpad = mpad_of(p);
  t.L = sys.L;
  t.h = sys.L / nc;
  for (int i = 0; i < 3; ++i) t.k[i] = sys.k[i];
  t.cplx = (sys.k[0] != 0.0 || sys.k[1] != 0.0 || sys.k[2] != 0.0);
  const double h = t.h;
  const int n = t.n;

  // ---- 1D tables: GLL basis, (p+1)-point Gauss quadrature (exact for the
  // stiffness, mass and derivative integrands on affine cells).
  std::vector<double> xi, wl, gq, gw;
  gll_rule(p, xi, wl);
  gauss_rule(p + 1, gq, gw);
  std::vector<double> K1(q * q, 0.0), Mc(q * q, 0.0), G1(q * q, 0.0);
  std::vector<double> l, dl;
  t.interp.assign(static_cast<size_t>(q) * q, 0.0);
  for (int iq = 0; iq <= p; ++iq) {
    lagrange_at(xi, gq[iq], l, dl);
    for (int a = 0; a < q; ++a) t.interp[iq * q + a] = l[a];
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b) {
        K1[a * q + b] += gw[iq] * (2.0 / h) * dl[a] * dl[b];
        Mc[a * q + b] += gw[iq] * (h / 2.0) * l[a] * l[b];
        G1[a * q + b] += gw[iq] * l[a] * dl[b];
      }
  }
  t.K1d = K1;
  t.M1d = Mc;
  // Loewdin scale per 1D index: shared (vertex-type) nodes collect the lumped
  // mass w_0 h/2 from both neighbouring cells.
  std::vector<double> dd_loc(q), dd_glob(p);
  for (int a = 0; a < q; ++a) {
    const double m = (a == 0 || a == p) ? wl[0] * h : wl[a] * h / 2.0;
    dd_loc[a] = 1.0 / std::sqrt(m);
  }
  for (int i = 0; i < p; ++i) dd_glob[i] = dd_loc[i];

  // ---- reference cell matrix A_k = D_c (K^c/2 - i skew(k.G^c)/2) D_c
  const int mc = t.mcell;
  t.cell_re.assign(static_cast<size_t>(mc) * mc, 0.0);
  if (t.cplx) t.cell_im.assign(static_cast<size_t>(mc) * mc, 0.0);
  std::vector<double> Dc(mc);
  for (int l0 = 0; l0 < mc; ++l0) {
    const int a = l0 % q, b = (l0 / q) % q, c = l0 / (q * q);
    Dc[l0] = dd_loc[a] * dd_loc[b] * dd_loc[c];
  }
  auto kG = [&](int l0, int l1) {
    const int a = l0 % q, b = (l0 / q) % q, c = l0 / (q * q);
    const int a1 = l1 % q, b1 = (l1 / q) % q, c1 = l1 / (q * q);
    return t.k[0] * G1[a * q + a1] * Mc[b * q + b1] * Mc[c * q + c1] +
           t.k[1] * Mc[a * q + a1] * G1[b * q + b1] * Mc[c * q + c1] +
           t.k[2] * Mc[a * q + a1] * Mc[b * q + b1] * G1[c * q + c1];
  };
  for (int l0 = 0; l0 < mc; ++l0) {
    const int a = l0 % q, b = (l0 / q) % q, c = l0 / (q * q);
    for (int l1 = 0; l1 < mc; ++l1) {
      const int a1 = l1 % q, b1 = (l1 / q) % q, c1 = l1 / (q * q);
      const double K = K1[a * q + a1] * Mc[b * q + b1] * Mc[c * q + c1] +
                       Mc[a * q + a1] * K1[b * q + b1] * Mc[c * q + c1] +
                       Mc[a * q + a1] * Mc[b * q + b1] * K1[c * q + c1];
      t.cell_re[static_cast<size_t>(l0) * mc + l1] = Dc[l0] * 0.5 * K * Dc[l1];
      if (t.cplx)
        t.cell_im[static_cast<size_t>(l0) * mc + l1] =
            -0.5 * Dc[l0] * (kG(l0, l1) - kG(l1, l0)) * Dc[l1];
    }
  }

  // ---- node coordinates, Loewdin scale, nodal potential
  t.x1d.resize(n);
  for (int i = 0; i < n; ++i) t.x1d[i] = (i / p) * h + (1.0 + xi[i % p]) * h / 2.0;
  t.dscale.resize(t.M);
  for (int64_t j = 0; j < t.M; ++j) {
    const int ix = static_cast<int>(j % n), iy = static_cast<int>((j / n) % n),
              iz = static_cast<int>(j / (static_cast<int64_t>(n) * n));
    t.dscale[j] = dd_glob[ix % p] * dd_glob[iy % p] * dd_glob[iz % p];
  }
  const double half_k2 = 0.5 * (t.k[0] * t.k[0] + t.k[1] * t.k[1] + t.k[2] * t.k[2]);
  t.vdiag.assign(t.M, half_k2);
  const double L = sys.L;
  // candidate 1D indices within `rc` of coordinate `center`
  auto near = [&](double center, double rc, std::vector<int>& out) {
    out.clear();
    for (int i = 0; i < n; ++i)
      if (std::fabs(t.x1d[i] - center) <= rc) out.push_back(i);
  };
  std::vector<int> cx, cy, cz;
  for (int at = 0; at < sys.natoms; ++at) {
    const double* R = sys.pos + 3 * at;
    const double s = sys.s[at], Z = sys.Z[at], rc = 10.0 * s;
    const int K = static_cast<int>(std::ceil(rc / L)) + 1;
    for (int nz = -K; nz <= K; ++nz)
      for (int ny = -K; ny <= K; ++ny)
        for (int nx = -K; nx <= K; ++nx) {
          const double sx = R[0] + nx * L, sy = R[1] + ny * L, sz = R[2] + nz * L;
          near(sx, rc, cx);
          near(sy, rc, cy);
          near(sz, rc, cz);
          for (int iz : cz)
            for (int iy : cy)
              for (int ix : cx) {
                const double dx = t.x1d[ix] - sx, dy = t.x1d[iy] - sy, dz = t.x1d[iz] - sz;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 > rc * rc) continue;
                t.vdiag[ix + static_cast<int64_t>(n) * (iy + static_cast<int64_t>(n) * iz)] +=
                    -Z * std::exp(-r2 / (2.0 * s * s));
              }
        }
  }

  t.atoms.assign(static_cast<size_t>(sys.natoms) * 8, 0.0);
  for (int at = 0; at < sys.natoms; ++at) {
    double* d = &t.atoms[static_cast<size_t>(at) * 8];
    d[0] = sys.pos[3 * at];
    d[1] = sys.pos[3 * at + 1];
    d[2] = sys.pos[3 * at + 2];
    d[3] = sys.Z[at];
    d[4] = sys.s[at];
    d[5] = (sys.has_proj && sys.h_s) ? sys.h_s[at] : 0.0;
    d[6] = (sys.has_proj && sys.h_p) ? sys.h_p[at] : 0.0;
  }

  // ---- projectors: c~_j = M_jj^(1/2) sum_images e^{-i k.(x_j - nL)} chi(x_j - R - nL)
  t.natoms = sys.natoms;
  t.has_proj = sys.has_proj != 0 && sys.natoms > 0;
  t.atom_ptr.assign(1, 0);
  t.atom_node.clear();
  t.atom_val.clear();
  t.pair_ptr.assign(t.E + 1, 0);
  t.pair_atom.clear();
  t.pair_re.clear();
  t.pair_im.clear();
  t.hcoef.assign(4 * sys.natoms, 0.0);
  if (!t.has_proj) return "";
  const int vw = t.cplx ? 8 : 4;
  using cd = std::complex<double>;
  struct Entry { int64_t node; cd v[4]; };
  struct PairRec { int64_t cell; int atom; std::vector<double> cre, cim; };
  std::vector<PairRec> pairs;
  std::vector<Entry> ent;
  for (int at = 0; at < sys.natoms; ++at) {
    const double w = sys.w[at];
    const double ns = 1.0 / std::sqrt(std::pow(M_PI, 1.5) * w * w * w);
    const double np_ = 1.0 / std::sqrt(std::pow(M_PI, 1.5) * std::pow(w, 5) / 2.0);
    const double rc = 6.0 * w;
    t.hcoef[4 * at] = sys.h_s[at];
    t.hcoef[4 * at + 1] = t.hcoef[4 * at + 2] = t.hcoef[4 * at + 3] = sys.h_p[at];
    const double* R = sys.pos + 3 * at;
    const int K = static_cast<int>(std::ceil(rc / L)) + 1;
    ent.clear();
    for (int nz = -K; nz <= K; ++nz)
      for (int ny = -K; ny <= K; ++ny)
        for (int nx = -K; nx <= K; ++nx) {
          const double shx = nx * L, shy = ny * L, shz = nz * L;
          const double sx = R[0] + shx, sy = R[1] + shy, sz = R[2] + shz;
          near(sx, rc, cx);
          near(sy, rc, cy);
          near(sz, rc, cz);
          for (int iz : cz)
            for (int iy : cy)
              for (int ix : cx) {
                const double dx = t.x1d[ix] - sx, dy = t.x1d[iy] - sy, dz = t.x1d[iz] - sz;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 > rc * rc) continue;
                const int64_t j = ix + static_cast<int64_t>(n) * (iy + static_cast<int64_t>(n) * iz);
                const double g = std::exp(-r2 / (2.0 * w * w)) / t.dscale[j];  // * M_jj^(1/2)
                cd ph(1.0, 0.0);
                if (t.cplx) {
                  const double arg = t.k[0] * (t.x1d[ix] - shx) + t.k[1] * (t.x1d[iy] - shy) +
                                     t.k[2] * (t.x1d[iz] - shz);
                  ph = cd(std::cos(arg), -std::sin(arg));
                }
                Entry e;
                e.node = j;
                e.v[0] = ph * (ns * g);
                e.v[1] = ph * (np_ * dx * g);
                e.v[2] = ph * (np_ * dy * g);
                e.v[3] = ph * (np_ * dz * g);
                ent.push_back(e);
              }
        }
    std::sort(ent.begin(), ent.end(), [](const Entry& a, const Entry& b) { return a.node < b.node; });
    // merge overlapping images, append to the atom-major list
    std::unordered_map<int64_t, size_t> cell_pair;
    for (size_t i = 0; i < ent.size();) {
      Entry e = ent[i];
      size_t j = i + 1;
      while (j < ent.size() && ent[j].node == e.node) {
        for (int m = 0; m < 4; ++m) e.v[m] += ent[j].v[m];
        ++j;
      }
      i = j;
      t.atom_node.push_back(static_cast<int32_t>(e.node));
      for (int m = 0; m < 4; ++m) {
        if (t.cplx) {
          t.atom_val.push_back(e.v[m].real());
          t.atom_val.push_back(e.v[m].imag());
        } else {
          t.atom_val.push_back(e.v[m].real());
        }
      }
      // the cells holding this node, with its local index and multiplicity
      const int ix = static_cast<int>(e.node % n), iy = static_cast<int>((e.node / n) % n),
                iz = static_cast<int>(e.node / (static_cast<int64_t>(n) * n));
      int cxs[2], axs[2], ncx = 0, cys[2], ays[2], ncy = 0, czs[2], azs[2], ncz = 0;
      auto cells_of = [&](int i1, int* cs, int* as, int& cnt) {
        cnt = 0;
        cs[cnt] = i1 / p; as[cnt] = i1 % p; ++cnt;
        if (i1 % p == 0) { cs[cnt] = (i1 / p - 1 + nc) % nc; as[cnt] = p; ++cnt; }
      };
      cells_of(ix, cxs, axs, ncx);
      cells_of(iy, cys, ays, ncy);
      cells_of(iz, czs, azs, ncz);
      const double inv_mult = 1.0 / (ncx * ncy * ncz);
      for (int uz = 0; uz < ncz; ++uz)
        for (int uy = 0; uy < ncy; ++uy)
          for (int ux = 0; ux < ncx; ++ux) {
            const int64_t cell = cxs[ux] + static_cast<int64_t>(nc) * (cys[uy] + static_cast<int64_t>(nc) * czs[uz]);
            const int lid = axs[ux] + q * (ays[uy] + q * azs[uz]);
            auto it = cell_pair.find(cell);
            size_t pi;
            if (it == cell_pair.end()) {
              pi = pairs.size();
              cell_pair.emplace(cell, pi);
              PairRec pr;
              pr.cell = cell;
              pr.atom = at;
              pr.cre.assign(static_cast<size_t>(mc) * 4, 0.0);
              if (t.cplx) pr.cim.assign(static_cast<size_t>(mc) * 4, 0.0);
              pairs.push_back(std::move(pr));
            } else {
              pi = it->second;
            }
            for (int m = 0; m < 4; ++m) {
              pairs[pi].cre[lid * 4 + m] = e.v[m].real() * inv_mult;
              if (t.cplx) pairs[pi].cim[lid * 4 + m] = e.v[m].imag() * inv_mult;
            }
          }
    }
    t.atom_ptr.push_back(static_cast<int64_t>(t.atom_node.size()));
  }
  (void)vw;
  // pairs sorted by (cell, atom), cell-major CSR, MFMA A-operand layout:
  // lane -> (row lane%16 of the row tile, projector component lane/16)
  std::vector<size_t> ord(pairs.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
    return pairs[a].cell != pairs[b].cell ? pairs[a].cell < pairs[b].cell : pairs[a].atom < pairs[b].atom;
  });
  const int rts = t.mpad / 16;
  t.pair_atom.resize(pairs.size());
  t.pair_re.assign(pairs.size() * rts * 64, 0.0);
  if (t.cplx) t.pair_im.assign(pairs.size() * rts * 64, 0.0);
  for (size_t k2 = 0; k2 < ord.size(); ++k2) {
    const PairRec& pr = pairs[ord[k2]];
    t.pair_atom[k2] = pr.atom;
    t.pair_ptr[pr.cell + 1] += 1;
    for (int rt = 0; rt < rts; ++rt)
      for (int lane = 0; lane < 64; ++lane) {
        const int r = rt * 16 + lane % 16, m = lane / 16;
        if (r >= mc) continue;
        t.pair_re[(k2 * rts + rt) * 64 + lane] = pr.cre[r * 4 + m];
        if (t.cplx) t.pair_im[(k2 * rts + rt) * 64 + lane] = pr.cim[r * 4 + m];
      }
  }
  for (int64_t c = 0; c < t.E; ++c) t.pair_ptr[c + 1] += t.pair_ptr[c];
  return "";
}

}  // namespace chfsi
