"""A small self-consistent field loop around the eigensolver, FP64
reference (the SCF procedure of Section 3, Algorithm 1, reduced to what a
synthetic system needs).

Test infrastructure only (see the package docstring).

Each step, in the paper's order:

* total electrostatic potential: the periodic Poisson problem
  -lap v_H = 4 pi (rho - rho_bar) in the FE basis, K v = 4 pi M (rho - rho_bar)
  (K the assembled stiffness, M the lumped mass, rho_bar the mean charge so
  that the right-hand side is neutral), with the constant fixed by
  sum_j M_jj v_j = 0; solved here exactly (sparse LU of the bordered
  system), the paper's solver being a Jacobi-preconditioned CG;
* exchange-correlation: LDA exchange only, v_x = -(3 rho / pi)^(1/3) (the
  XC functional is not the point here; the paper uses GGA through libxc);
* effective potential V = V_ext + v_H + v_x on the nodes (the nodal
  potential of ``fe.build_operator``); the discrete Hamiltonian with it;
* eigenpairs of the N lowest states (dense eigh: the fixed point does not
  depend on the eigensolver);
* Fermi level and occupations, the nodal density (``density``);
* density mixing: Anderson's method on rho with M-weighted inner products.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import density as dens
from . import fe


def stiffness(op: fe.Operator) -> sp.csr_matrix:
    """Assembled FE stiffness K (no Loewdin scaling)."""
    E, mc = op.cells.shape
    rows = np.repeat(op.cells, mc, axis=1).ravel()
    cols = np.tile(op.cells, (1, mc)).ravel()
    return sp.csr_matrix((np.tile(op.ct.K.ravel(), E), (rows, cols)), shape=(op.M, op.M))


def hartree(op: fe.Operator, rho: np.ndarray) -> np.ndarray:
    """v_H with K v = 4 pi M (rho - rho_bar), sum M v = 0."""
    m = op.Mdiag
    rho_bar = float(np.sum(m * rho) / np.sum(m))
    b = 4.0 * np.pi * m * (rho - rho_bar)
    K = stiffness(op)
    A = sp.bmat([[K, sp.csr_matrix(m[:, None])], [sp.csr_matrix(m[None, :]), None]], format="csc")
    sol = spla.spsolve(A, np.concatenate([b, [0.0]]))
    return sol[:-1]


def lda_exchange(rho: np.ndarray) -> np.ndarray:
    return -np.cbrt(3.0 * np.maximum(rho, 0.0) / np.pi)


def hamiltonian(op: fe.Operator, V: np.ndarray) -> np.ndarray:
    return fe.dense(dataclasses.replace(op, V=V, _A0=None, _asm=None))


class Anderson:
    """Anderson mixing x_{n+1} = xbar + beta Fbar with xbar = x - dX g,
    Fbar = F - dF g, g minimising |F - dF g|_W (W-weighted norm), over the
    last ``depth`` differences."""

    def __init__(self, beta: float, depth: int, weight: np.ndarray):
        self.beta, self.depth, self.w = beta, depth, weight
        self.xs: List[np.ndarray] = []
        self.fs: List[np.ndarray] = []

    def step(self, x: np.ndarray, F: np.ndarray) -> np.ndarray:
        self.xs.append(x.copy())
        self.fs.append(F.copy())
        if len(self.xs) > self.depth + 1:
            self.xs.pop(0)
            self.fs.pop(0)
        if len(self.xs) == 1:
            return x + self.beta * F
        dX = np.stack([self.xs[i + 1] - self.xs[i] for i in range(len(self.xs) - 1)], axis=1)
        dF = np.stack([self.fs[i + 1] - self.fs[i] for i in range(len(self.fs) - 1)], axis=1)
        A = dF.T @ (self.w[:, None] * dF)
        r = dF.T @ (self.w * F)
        g = np.linalg.lstsq(A, r, rcond=None)[0]
        return (x - dX @ g) + self.beta * (F - dF @ g)


@dataclasses.dataclass
class SCFResult:
    rho: np.ndarray
    V: np.ndarray
    theta: np.ndarray
    mu: float
    residuals: List[float]
    converged: bool


def scf(sys, nstates: int, n_electrons: float, kT: float, beta: float = 0.3, depth: int = 4,
        tol: float = 1e-8, maxit: int = 60, rho0: Optional[np.ndarray] = None) -> SCFResult:
    op = fe.build_operator(sys)
    m = op.Mdiag
    V_ext = op.V.copy()
    rho = np.full(op.M, n_electrons / float(np.sum(m))) if rho0 is None else rho0.copy()
    mix = Anderson(beta, depth, m)
    res: List[float] = []
    th = np.zeros(nstates)
    mu = 0.0
    V = V_ext
    for _ in range(maxit):
        V = V_ext + hartree(op, rho) + lda_exchange(rho)
        lam, U = np.linalg.eigh(hamiltonian(op, V))
        th = lam[:nstates]
        mu = dens.fermi_level(th, n_electrons, kT)
        f = dens.occupations(th, mu, kT)
        rho_out = dens.density(U[:, :nstates], 2.0 * f, m)
        F = rho_out - rho
        res.append(float(np.sqrt(np.sum(m * F * F))))
        if res[-1] < tol:
            return SCFResult(rho_out, V, th, mu, res, True)
        rho = mix.step(rho, F)
    return SCFResult(rho, V, th, mu, res, False)
