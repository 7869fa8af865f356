// Per-cell local potential by Gauss quadrature: the discrete Hamiltonian
// construction of Section 4.2 (Eq. quadLocal, Eq. gemmLoc).
//
//   K^loc_e[j, k] = sum_q N_j(x_q) N_k(x_q) V(x_q) w_q |J|
//
// for all cells at once is one product P V~ with P[(j,k), q] = N_j(x_q) N_k(x_q)
// over the pairs j <= k (M_sym = mcell (mcell + 1) / 2 rows) and
// V~[q, e] = V(x_q^e) w_q |J|.  The product is a plain dense GEMM
// (rocBLAS).  These kernels build V~ on the device and expand the packed
// result into per-cell matrices in the MFMA A-operand order the cell kernel
// reads: A_e = A_shared + D_c K^loc_e D_c, where A_shared already holds
// D_c (K^c / 2) D_c.
#include "internal.h"

namespace chfsi {
namespace {

// V~[e * nq + q]: Gaussian-atom potential at the Gauss point q of cell e
// times the point's weight and the Jacobian.  Periodic images: every shift n
// with |x_i - R_i - n_i L| <= 10 s per axis and r <= 10 s (the image rule of
// the nodal potential).
__global__ void __launch_bounds__(256)
gauss_potential_kernel(const double* __restrict__ atoms, int natoms, double L, int nc, int p,
                       const double* __restrict__ gq, const double* __restrict__ gw, double jac,
                       double* __restrict__ Vw) {
  const int q1 = p + 1, nq = q1 * q1 * q1;
  const int64_t E = static_cast<int64_t>(nc) * nc * nc;
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= E * nq) return;
  const int64_t e = idx / nq;
  const int qp = static_cast<int>(idx % nq);
  const int qx = qp % q1, qy = (qp / q1) % q1, qz = qp / (q1 * q1);
  const int cx = static_cast<int>(e % nc), cy = static_cast<int>((e / nc) % nc), cz = static_cast<int>(e / (nc * nc));
  const double h = L / nc;
  const double x[3] = {cx * h + (1.0 + gq[qx]) * h * 0.5, cy * h + (1.0 + gq[qy]) * h * 0.5,
                       cz * h + (1.0 + gq[qz]) * h * 0.5};
  double v = 0.0;
  for (int a = 0; a < natoms; ++a) {
    const double* at = atoms + 8 * a;
    const double Z = at[3], s = at[4], rc = 10.0 * s;
    int lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
      const double d = x[i] - at[i];
      lo[i] = static_cast<int>(ceil((d - rc) / L));
      hi[i] = static_cast<int>(floor((d + rc) / L));
    }
    for (int nz = lo[2]; nz <= hi[2]; ++nz)
      for (int ny = lo[1]; ny <= hi[1]; ++ny)
        for (int nx = lo[0]; nx <= hi[0]; ++nx) {
          const double dx = x[0] - at[0] - nx * L, dy = x[1] - at[1] - ny * L, dz = x[2] - at[2] - nz * L;
          if (fabs(dx) > rc || fabs(dy) > rc || fabs(dz) > rc) continue;
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 <= rc * rc) v += -Z * exp(-r2 / (2.0 * s * s));
        }
  }
  Vw[idx] = v * gw[qx] * gw[qy] * gw[qz] * jac;
}

// A_e[(rt * KS + ks) * 64 + lane] = A_shared[same] + D_i D_k K^loc_e[pair(i, k)]
// with i = 16 rt + lane % 16, k = 4 ks + lane / 16 (padding rows and
// columns copy the shared matrix's zeros).  pair(j, k), j <= k, is the
// row j * mcell - j (j - 1) / 2 + (k - j) of the packed product.
__global__ void __launch_bounds__(256)
assemble_cell_matrices_kernel(const double* __restrict__ Ash, const double* __restrict__ Kloc, int64_t msym,
                              const double* __restrict__ Dl, int mcell, int mpad, int64_t E,
                              double* __restrict__ Ae) {
  const int64_t per = static_cast<int64_t>(mpad) * mpad;
  const int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (idx >= E * per) return;
  const int64_t e = idx / per;
  const int o = static_cast<int>(idx % per);
  const int KS = mpad / 4;
  const int lane = o % 64, tile = o / 64;
  const int rt = tile / KS, ks = tile % KS;
  const int i = rt * 16 + lane % 16, k = ks * 4 + lane / 16;
  double v = Ash[o];
  if (i < mcell && k < mcell) {
    const int j0 = i < k ? i : k, j1 = i < k ? k : i;
    const int64_t pr = static_cast<int64_t>(j0) * mcell - static_cast<int64_t>(j0) * (j0 - 1) / 2 + (j1 - j0);
    v += Dl[i] * Dl[k] * Kloc[e * msym + pr];
  }
  Ae[idx] = v;
}

unsigned blocks_of(int64_t total) { return static_cast<unsigned>((total + 255) / 256); }

}  // namespace

hipError_t launch_gauss_potential(const double* atoms, int natoms, double L, int nc, int p, const double* gq,
                                  const double* gw, double* Vw, hipStream_t s) {
  const int64_t total = static_cast<int64_t>(nc) * nc * nc * (p + 1) * (p + 1) * (p + 1);
  const double h = L / nc;
  const double jac = (h / 2.0) * (h / 2.0) * (h / 2.0);
  hipLaunchKernelGGL(gauss_potential_kernel, dim3(blocks_of(total)), dim3(256), 0, s, atoms, natoms, L, nc, p, gq,
                     gw, jac, Vw);
  return hipGetLastError();
}

hipError_t launch_assemble_cell_matrices(const double* Ash, const double* Kloc, int64_t msym, const double* Dl,
                                         int mcell, int mpad, int64_t E, double* Ae, hipStream_t s) {
  const int64_t total = E * mpad * static_cast<int64_t>(mpad);
  if (blocks_of(total) == 0 || (total + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(assemble_cell_matrices_kernel, dim3(blocks_of(total)), dim3(256), 0, s, Ash, Kloc, msym, Dl,
                     mcell, mpad, E, Ae);
  return hipGetLastError();
}

}  // namespace chfsi
