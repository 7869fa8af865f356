"""Per-cell local potential by Gauss quadrature (the discrete-Hamiltonian
construction of Section 4.2), FP64 reference.

Test infrastructure only (see the package docstring).

In the operator of ``fe.build_operator`` the local potential is collocated
at the GLL nodes (a diagonal term).  Here it is integrated the way the
paper's cell-level Hamiltonian does it: for every cell e,

    K^loc_e[a, b] = sum_q N_a(x_q) N_b(x_q) V(x_q) w_q |J|

over the (p+1)^3 Gauss-Legendre points of the cell (Eq. quadLocal), which
the paper evaluates for all cells at once as one product of the matrix of
basis-function products (pairs a <= b by points) with the matrix of
quadrature-weighted potential values (points by cells) (Eq. gemmLoc).  The
Loewdin-transformed operator is then

    H~ = D (K/2 - i k.G) D + D (sum_e K^loc_e) D + |k|^2/2 + H~_nl

with the same lumped D = M^-1/2 and the same nonlocal part as before; the
constant |k|^2/2 stays on the lumped diagonal.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fe


def gauss_points_1d(ncell: int, p: int, L: float) -> np.ndarray:
    """Coordinates of the (p+1) Gauss points of every cell along one axis,
    cell-major: index c (p+1) + q."""
    h = L / ncell
    gq, _ = fe.gauss_legendre(p + 1)
    return (np.arange(ncell)[:, None] * h + (1.0 + gq[None, :]) * h / 2.0).ravel()


def gauss_potential(sys) -> np.ndarray:
    """(E, (p+1)^3): V at the Gauss points of every cell (cell id
    cx + nc (cy + nc cz), point qx + (p+1)(qy + (p+1) qz)), the same
    Gaussian-atom potential as the nodal one."""
    nc, q = sys.ncell, sys.p + 1
    g1 = gauss_points_1d(nc, sys.p, sys.L)
    V = fe.local_potential(sys, g1).reshape(nc, q, nc, q, nc, q)    # [cz, qz, cy, qy, cx, qx]
    V = V.transpose(0, 2, 4, 1, 3, 5)                                # [cz, cy, cx, qz, qy, qx]
    return V.reshape(nc ** 3, q ** 3)


def basis_at_gauss(p: int) -> np.ndarray:
    """N[q, a]: the cell's GLL Lagrange basis functions at its Gauss points."""
    xi, _ = fe.gll(p)
    gq, _ = fe.gauss_legendre(p + 1)
    L1, _ = fe.lagrange(xi, gq)
    return fe.kron3(L1, L1, L1)


def cell_local_matrices(sys, Vq: np.ndarray) -> np.ndarray:
    """(E, mcell, mcell) K^loc_e from the Gauss-point potential Vq (E, nq)."""
    p, h = sys.p, sys.L / sys.ncell
    _, gw = fe.gauss_legendre(p + 1)
    W = fe.kron3(gw, gw, gw) * (h / 2.0) ** 3
    N = basis_at_gauss(p)
    return np.einsum("qa,eq,qb->eab", N, Vq * W[None, :], N, optimize=True)


def assemble_quadrature(sys, k=None) -> sp.csr_matrix:
    """Sparse H~(k) with the local potential integrated per cell."""
    op = fe.build_operator(sys, k)
    Vq = gauss_potential(sys) if sys.natoms else np.zeros((op.E, (sys.p + 1) ** 3))
    Kl = cell_local_matrices(sys, Vq)
    E, mc = op.cells.shape
    rows = np.repeat(op.cells, mc, axis=1).ravel()
    cols = np.tile(op.cells, (1, mc)).ravel()
    Kloc = sp.csr_matrix((Kl.ravel(), (rows, cols)), shape=(op.M, op.M))
    K = sp.csr_matrix((np.tile(op.ct.K.ravel(), E), (rows, cols)), shape=(op.M, op.M))
    H = 0.5 * K + Kloc
    if op.is_complex:
        for al in range(3):
            if op.k[al] != 0.0:
                G = sp.csr_matrix((np.tile(op.ct.G[al].ravel(), E), (rows, cols)), shape=(op.M, op.M))
                H = H - 1j * op.k[al] * G
    Dm = sp.diags(op.D)
    H = Dm @ H @ Dm + 0.5 * float(op.k @ op.k) * sp.identity(op.M)
    if op.C is not None:
        H = H + op.C @ sp.diags(op.hvec) @ op.C.conj().T
    return sp.csr_matrix(H)
