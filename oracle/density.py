"""Electron density at the nodes and the Fermi level, FP64 reference.

Test infrastructure only (see the package docstring).

What is computed, and where the paper defines it (Section 3.2, the density
computation algorithm, and the Fermi-Dirac occupations of Section 2.1):

* Occupations f_i = 1 / (1 + exp((theta_i - mu) / kT)) of the Ritz values,
  with the Fermi level mu fixed by the electron count,
  2 sum_i w_i f_i = N_e (spin factor 2, optional k-point weights w_i).
* The density at the (p+1)^3 Gauss-Legendre points of every cell (the
  algorithm evaluates it inside each cell through the cell's FE basis
  functions): psi^ restricted to the cell is interpolated with the
  tensor-product Lagrange basis on the GLL nodes, then squared and weighted.
* The density at a node x_j of the spectral mesh.  The FE basis function of
  node j is 1 at x_j and 0 at every other node, so n(x_j) = e_j and the
  density algorithm reduces to
  rho(x_j) = 2 sum_i f_i |psi^_i(x_j)|^2,  psi^ = M^-1/2 psi~,
  i.e. rho_j = (1 / M_jj) sum_i w'_i |Psi~_{j,i}|^2 with w'_i = 2 f_i.
  The algorithm's spectrum-split form (an orthonormal basis of the filtered
  space with weight 2, plus the fractionally occupied Ritz vectors with
  weight 2 (f_i - 1)) is the same sum written with other vectors; both are
  weighted sums of squared moduli, which is what ``density`` evaluates.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import fe


def occupations(theta: np.ndarray, mu: float, kT: float) -> np.ndarray:
    """Fermi-Dirac occupations, evaluated without overflow."""
    x = (np.asarray(theta, dtype=np.float64) - mu) / kT
    out = np.empty_like(x)
    pos = x > 0
    e = np.exp(-x[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def electron_count(theta, mu: float, kT: float, weights: Optional[np.ndarray] = None) -> float:
    f = occupations(theta, mu, kT)
    w = np.ones_like(f) if weights is None else np.asarray(weights, dtype=np.float64)
    return float(2.0 * np.sum(w * f))


def fermi_level(theta, n_electrons: float, kT: float, weights: Optional[np.ndarray] = None,
                iters: int = 200) -> float:
    """mu with 2 sum_i w_i f((theta_i - mu)/kT) = n_electrons, by bisection
    (the count is increasing in mu)."""
    theta = np.asarray(theta, dtype=np.float64)
    total = 2.0 * (len(theta) if weights is None else float(np.sum(weights)))
    if not (0.0 < n_electrons < total):
        raise ValueError("electron count must lie strictly between 0 and 2 sum(w)")
    lo, hi = theta.min() - 50.0 * kT, theta.max() + 50.0 * kT
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if electron_count(theta, mid, kT, weights) < n_electrons:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def density(Psi: np.ndarray, w: np.ndarray, Mdiag: np.ndarray) -> np.ndarray:
    """rho_j = (1 / M_jj) sum_c w_c |Psi_{j,c}|^2 for the Loewdin-basis block
    Psi (M x ncols, real or complex)."""
    Psi = np.asarray(Psi)
    s = (np.abs(Psi) ** 2) @ np.asarray(w, dtype=np.float64)
    return s / np.asarray(Mdiag, dtype=np.float64)


def density_gauss_cell(p: int, Ph_e: np.ndarray, w: np.ndarray) -> np.ndarray:
    """rho at the (p+1)^3 Gauss points of one cell from the cell's scaled
    nodal values Ph_e (mcell x ncols, psi^ = M^-1/2 psi~, local node order
    a + (p+1)(b + (p+1) c)).  Point order qx + (p+1)(qy + (p+1) qz)."""
    xi, _ = fe.gll(p)
    gq, _ = fe.gauss_legendre(p + 1)
    L1, _ = fe.lagrange(xi, gq)          # L1[q, a] = l_a(g_q)
    N = fe.kron3(L1, L1, L1)              # N[point, node]
    vals = N @ Ph_e
    return (np.abs(vals) ** 2) @ np.asarray(w, dtype=np.float64)


def density_gauss(ncell: int, p: int, L: float, Psi: np.ndarray, w: np.ndarray,
                  cells: Optional[np.ndarray] = None) -> np.ndarray:
    """rho[e, point] for the listed cells (default all), cell id
    cx + ncell (cy + ncell cz)."""
    Mdiag = fe.lumped_mass(ncell, p, L)
    D = 1.0 / np.sqrt(Mdiag)
    nodes = fe.cell_nodes(ncell, p)
    ids = np.arange(nodes.shape[0]) if cells is None else np.asarray(cells)
    out = np.empty((ids.size, (p + 1) ** 3))
    for i, e in enumerate(ids):
        rows = nodes[e]
        out[i] = density_gauss_cell(p, D[rows, None] * Psi[rows], w)
    return out
