"""Rayleigh-Ritz through the generalised eigenproblem with spectrum
splitting, and its mixed-precision form: FP64 reference.

Test infrastructure only (see the package docstring).

Algorithm 2 of Section 3.2, in its order, on the filtered block Psi_f
(M x N, not orthonormal):

* RRGEP-O   S = Psi_f^H Psi_f
* RRGEP-P   H^ = Psi_f^H H~ Psi_f
* RRGEP-D   S = L L^H (Cholesky); the generalised problem H^ Q = S Q D is
            recast as the standard one (L^-1 H^ L^-H) Q' = Q' D with
            Q = L^-H Q'; only the N_fr highest pairs are kept for vectors
            (all N eigenvalues are returned, they cost nothing extra here)
* RRGEP-ST-F  Psi^R_fr = Psi_f Q_fr   (the fractionally occupied Ritz vectors)
* RRGEP-ST-O  Psi_o = Psi_f L^-H      (orthonormal basis of the span)

Mixed precision (Section 3.2 and the Rayleigh-Ritz part of Section 4.4):
diagonal blocks of S (block width ``block``) in FP64, off-diagonal blocks in
FP32; H^ in FP32 except its fr-fr block (the last N_fr rows and columns),
which is FP64; Psi_o = FP32[Psi_f (L^-H with its diagonal removed)] +
FP64[Psi_f diag(L^-H)].  "FP32" here means both factors rounded to float32
and the product formed in float32 arithmetic (numpy's float32 matmul).
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np
import scipy.linalg as sla

Apply = Callable[[np.ndarray], np.ndarray]


@dataclasses.dataclass
class RRGEPResult:
    theta: np.ndarray      # all N eigenvalues of H^ Q = S Q D, ascending
    psi_fr: np.ndarray     # M x N_fr: Psi_f Q_fr (the N_fr highest)
    psi_o: np.ndarray      # M x N: Psi_f L^-H
    Q: np.ndarray          # N x N: all generalised eigenvectors, L^-H Q'
    L: np.ndarray          # N x N lower Cholesky factor of S


def _ah(A):
    return A.conj().T


def _prod32(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A B with both factors rounded to single precision and the product
    formed in single precision, returned in double."""
    ct = np.complex64 if (np.iscomplexobj(A) or np.iscomplexobj(B)) else np.float32
    return (A.astype(ct) @ B.astype(ct)).astype(np.complex128 if ct == np.complex64 else np.float64)


def overlap(Psi: np.ndarray, mixed: bool, block: int) -> np.ndarray:
    """RRGEP-O: S = Psi^H Psi (mixed: off-diagonal blocks in FP32)."""
    S = _ah(Psi) @ Psi
    if mixed:
        N = Psi.shape[1]
        S32 = _prod32(_ah(Psi), Psi)
        for i0 in range(0, N, block):
            for j0 in range(0, N, block):
                if i0 != j0:
                    S[i0:i0 + block, j0:j0 + block] = S32[i0:i0 + block, j0:j0 + block]
    return S


def projected(Psi: np.ndarray, HPsi: np.ndarray, nfr: int, mixed: bool) -> np.ndarray:
    """RRGEP-P: H^ = Psi^H (H~ Psi) (mixed: all blocks but fr-fr in FP32)."""
    if not mixed:
        return _ah(Psi) @ HPsi
    N = Psi.shape[1]
    Hh = _prod32(_ah(Psi), HPsi)
    f0 = N - nfr
    Hh[f0:, f0:] = _ah(Psi[:, f0:]) @ HPsi[:, f0:]
    return Hh


def rrgep(apply: Apply, Psi: np.ndarray, nfr: int, mixed: bool = False, block: int = 128) -> RRGEPResult:
    N = Psi.shape[1]
    if not (1 <= nfr <= N):
        raise ValueError("1 <= nfr <= N")
    S = overlap(Psi, mixed, block)
    S = 0.5 * (S + _ah(S))
    Hh = projected(Psi, apply(Psi), nfr, mixed)
    Hh = 0.5 * (Hh + _ah(Hh))
    L = np.linalg.cholesky(S)
    Linv = sla.solve_triangular(L, np.eye(N), lower=True)
    Hs = Linv @ Hh @ _ah(Linv)
    Hs = 0.5 * (Hs + _ah(Hs))
    theta, Qp = np.linalg.eigh(Hs)
    Q = _ah(Linv) @ Qp
    psi_fr = Psi @ Q[:, N - nfr:]
    LinvH = _ah(Linv)
    if mixed:
        d = np.diag(LinvH).copy()
        off = LinvH - np.diag(d)
        psi_o = _prod32(Psi, off) + Psi * d[None, :]
    else:
        psi_o = Psi @ LinvH
    return RRGEPResult(theta, psi_fr, psi_o, Q, L)
