"""Chebyshev-filtered subspace iteration, FP64 reference.

Test infrastructure only (see the package docstring).

Steps, in the paper's order (Section 3.1 and Algorithm 2):

* ``lanczos_bound``  upper bound b of the spectrum from a k-step Lanczos
  run without reorthogonalisation, b = theta_max(T_k) + ||f_k|| (the
  estimator of Zhou and Li, 2011; the paper says only that the filter is
  built from an upper bound of H~).
* ``cheb_filter``    the degree-m Chebyshev filter of Section 3.1 applied
  to a block, with [a, b] mapped to [-1, 1] and the recurrence rescaled
  every step so that values stay of order one (same span as the
  unscaled three-term recurrence).
* ``cholgs``         RRGEP-O and the Cholesky factor of Algorithm 2:
  S = X^H X, S = L L^H, X_o = X L^-H.
* ``rayleigh_ritz``  RRGEP-P/D/ST on the orthonormal block: H^ = X_o^H H~ X_o
  (Hermitised), eigh, Psi = X_o Q', H~Psi, residual norms.
* ``solve``          bound, initial Rayleigh-Ritz, then passes of
  filter + CholGS + RR with a = largest and a_L = smallest Ritz value.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

Apply = Callable[[np.ndarray], np.ndarray]


def lanczos_bound(apply: Apply, v0: np.ndarray, steps: int = 20):
    """Return (b_upper, theta_min, theta_max, fnorm) from ``steps`` Lanczos steps."""
    v = np.asarray(v0).astype(np.result_type(v0.dtype, np.float64)).copy()
    v /= np.linalg.norm(v)
    alphas: List[float] = []
    betas: List[float] = []
    f = apply(v)
    alpha = float(np.real(np.vdot(v, f)))
    f = f - alpha * v
    alphas.append(alpha)
    v_prev = v
    for _ in range(1, steps):
        beta = float(np.linalg.norm(f))
        if beta == 0.0:
            break
        v = f / beta
        f = apply(v) - beta * v_prev
        alpha = float(np.real(np.vdot(v, f)))
        f = f - alpha * v
        alphas.append(alpha)
        betas.append(beta)
        v_prev = v
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    th = np.linalg.eigvalsh(T)
    fn = float(np.linalg.norm(f))
    return th[-1] + fn, th[0], th[-1], fn


def cheb_coeffs(m: int, a: float, b: float, aL: float):
    """Per-step scalars (alpha_i, beta_i) of the scaled recurrence.

    Step 1: Y = alpha_1 (H~X - cX).  Step i >= 2:
    Z = alpha_i (H~Y - cY) - beta_i X.  Returns (c, [(alpha_i, beta_i)]).
    """
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sigma1 = e / (aL - c)
    sigma = sigma1
    out = [(sigma1 / e, 0.0)]
    for _ in range(2, m + 1):
        sn = 1.0 / (2.0 / sigma1 - sigma)
        out.append((2.0 * sn / e, sigma * sn))
        sigma = sn
    return c, out


def cheb_filter(apply: Apply, X: np.ndarray, m: int, a: float, b: float, aL: float) -> np.ndarray:
    """Scaled degree-m Chebyshev filter: T_m(H_bar) X / T_m((aL - c)/e),
    H_bar = (H~ - c)/e, e = (b - a)/2, c = (b + a)/2."""
    if not (aL < a < b):
        raise ValueError("need aL < a < b")
    c, co = cheb_coeffs(m, a, b, aL)
    al, _ = co[0]
    Xp = X
    Y = al * (apply(X) - c * X)
    for i in range(1, m):
        al, be = co[i]
        Z = al * (apply(Y) - c * Y) - be * Xp
        Xp, Y = Y, Z
    return Y


def cheb_explicit(evals: np.ndarray, m: int, a: float, b: float, aL: float) -> np.ndarray:
    """T_m((lam - c)/e) / T_m((aL - c)/e) from the closed form of T_m
    (cos(m arccos t) inside [-1, 1], sign(t)^m cosh(m arccosh|t|) outside)."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0

    def T(t):
        t = np.asarray(t, dtype=np.float64)
        out = np.empty_like(t)
        inside = np.abs(t) <= 1.0
        out[inside] = np.cos(m * np.arccos(t[inside]))
        o = ~inside
        out[o] = np.sign(t[o]) ** m * np.cosh(m * np.arccosh(np.abs(t[o])))
        return out

    return T((evals - c) / e) / T(np.array([(aL - c) / e]))[0]


def cholgs(X: np.ndarray):
    """S = X^H X, L = chol(S) (lower), X_o = X L^-H.  Raises LinAlgError if
    S is not positive definite."""
    S = X.conj().T @ X
    Lc = np.linalg.cholesky(S)
    Xo = sla.solve_triangular(Lc.conj(), X.T, lower=True).T  # X L^-H
    return Xo, Lc, S


def rayleigh_ritz(apply: Apply, Xo: np.ndarray):
    """Returns (theta ascending, Psi, HPsi, residual norms, Hhat)."""
    W = apply(Xo)
    Hh = Xo.conj().T @ W
    Hh = 0.5 * (Hh + Hh.conj().T)
    th, Q = np.linalg.eigh(Hh)
    Psi = Xo @ Q
    HPsi = W @ Q
    r = np.linalg.norm(HPsi - Psi * th[None, :], axis=0)
    return th, Psi, HPsi, r, Hh


@dataclasses.dataclass
class SolveResult:
    theta: np.ndarray
    X: np.ndarray
    resid: np.ndarray
    passes: int
    b: float
    history: List[np.ndarray]
    resid_history: List[np.ndarray]
    bounds_history: List[tuple]


def solve(apply: Apply, X0: np.ndarray, nwanted: int, m: int, block: int,
          v0: np.ndarray, lanczos_steps: int = 20, passes: Optional[int] = None,
          tol: Optional[float] = None, max_passes: int = 200,
          b: Optional[float] = None) -> SolveResult:
    """Plain ChFSI: bound, initial CholGS + RR, then passes of
    (filter every column block, CholGS, RR) until ``passes`` are done or
    max_{i <= nwanted} r_i <= tol."""
    if b is None:
        b = lanczos_bound(apply, v0, lanczos_steps)[0]
    X = np.array(X0, copy=True)
    ncols = X.shape[1]
    Xo, _, _ = cholgs(X)
    th, X, _, r, _ = rayleigh_ritz(apply, Xo)
    hist = [th.copy()]
    rhist = [r.copy()]
    bh = []
    npass = 0
    limit = passes if passes is not None else max_passes
    while npass < limit:
        if passes is None and tol is not None and np.max(r[:nwanted]) <= tol:
            break
        a = float(th[ncols - 1])
        aL = float(th[0])
        bh.append((a, b, aL))
        Xf = np.empty_like(X)
        for c0 in range(0, ncols, block):
            Xf[:, c0:c0 + block] = cheb_filter(apply, X[:, c0:c0 + block], m, a, b, aL)
        Xo, _, _ = cholgs(Xf)
        th, X, _, r, _ = rayleigh_ritz(apply, Xo)
        hist.append(th.copy())
        rhist.append(r.copy())
        npass += 1
    return SolveResult(th[:nwanted], X[:, :nwanted], r[:nwanted], npass, b, hist, rhist, bh)


def subspace_sine(Psi: np.ndarray, Ref: np.ndarray) -> float:
    """Sine of the largest principal angle between span(Psi) and span(Ref)
    (both with orthonormal columns)."""
    P = Ref.conj().T @ Psi
    R = Psi - Ref @ P
    return float(np.linalg.norm(R, 2))
