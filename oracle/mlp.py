"""Learned warm start for ChFSI, FP64 reference.

Test infrastructure only (see the package docstring).  The paper has no
learned component; this is the spec extension whose readings are:

* Features (per node j, 32 values): 8 radial centres mu_k = k bohr
  (k = 0..7), width eta = 0.5 bohr, times 4 per-atom channels
  phi(a) in {Z_a, s_a, h_s,a, h_p,a}:
  f[j, 8 q + k] = sum_a sum_images phi_q(a) exp(-(r - mu_k)^2 / (2 eta^2)),
  r = |x_j - R_a - nL|, image terms with r <= 10 bohr.
* Network: 32 -> 128 (tanh) -> 128 (tanh) -> 128 (linear) on standardised
  features (f - mean) / std.
* Loss per configuration, with Y the output block and Q the converged
  orthonormal Ritz block (both M x 128):
  l = ||Y - Q Q^T Y||_F^2 / ||Y||_F^2 + 0.1 ||128 Y^T Y / ||Y||_F^2 - I||_F^2 / 128^2
      + (1 - tr(Q^T Y (Y^T Y + eps I)^-1 Y^T Q) / 128),   eps = 0.01 ||Y||_F^2 / 128
  (rotation, sign and scale invariant).  The first term is the part of the
  output outside the target subspace, the third the part of the target
  outside the output's span, ||Q - P_Y Q||_F^2 / 128 with the projector
  P_Y = Y (Y^T Y)^-1 Y^T regularised by a ridge of 1 % of the mean
  eigenvalue of Y^T Y (so that an output confined to a few target
  directions is penalised, and directions the output barely holds count
  only in proportion); the second keeps the columns from collapsing onto
  one direction.
* Adam (lr, beta1 = 0.9, beta2 = 0.999, eps = 1e-8).
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

MU = np.arange(8, dtype=np.float64)
ETA = 0.5
RCUT = 10.0


def features(sys, coords: np.ndarray) -> np.ndarray:
    """(M, 32) radial features of the nodes at ``coords`` (M x 3)."""
    L = sys.L
    M = coords.shape[0]
    F = np.zeros((M, 32))
    chans = [np.asarray(sys.Z), np.asarray(sys.s),
             np.asarray(sys.h_s) if sys.h_s is not None else np.zeros(sys.natoms),
             np.asarray(sys.h_p) if sys.h_p is not None else np.zeros(sys.natoms)]
    K = int(math.ceil(RCUT / L)) + 1
    for a in range(sys.natoms):
        for nz in range(-K, K + 1):
            for ny in range(-K, K + 1):
                for nx in range(-K, K + 1):
                    d = coords - (sys.pos[a] + L * np.array([nx, ny, nz], dtype=np.float64))
                    r = np.sqrt(np.sum(d * d, axis=1))
                    sel = r <= RCUT
                    if not np.any(sel):
                        continue
                    g = np.exp(-((r[sel, None] - MU[None, :]) ** 2) / (2.0 * ETA * ETA))  # (m, 8)
                    for q in range(4):
                        F[sel, 8 * q: 8 * q + 8] += chans[q][a] * g
    return F


def init_params(din: int, hidden: int, dout: int, rng: np.random.Generator) -> Dict[str, np.ndarray]:
    """Xavier-uniform weights, zero biases."""
    def xavier(fi, fo):
        lim = math.sqrt(6.0 / (fi + fo))
        return rng.uniform(-lim, lim, size=(fi, fo))
    return {"W1": xavier(din, hidden), "b1": np.zeros(hidden),
            "W2": xavier(hidden, hidden), "b2": np.zeros(hidden),
            "W3": xavier(hidden, dout), "b3": np.zeros(dout)}


def forward(params, Fn: np.ndarray):
    """Returns (Y, cache) for standardised features Fn (M x din)."""
    Z1 = Fn @ params["W1"] + params["b1"]
    A1 = np.tanh(Z1)
    Z2 = A1 @ params["W2"] + params["b2"]
    A2 = np.tanh(Z2)
    Y = A2 @ params["W3"] + params["b3"]
    return Y, (Fn, A1, A2)


def loss_and_grad_Y(Y: np.ndarray, Q: np.ndarray, lam: float = 0.1, mu: float = 1.0, delta: float = 0.01):
    """Subspace loss and its gradient with respect to Y."""
    n = Y.shape[1]
    nq = Q.shape[1]
    s = float(np.sum(Y * Y))
    P = Q.T @ Y
    R = Y - Q @ P
    r2 = float(np.sum(R * R))
    G = n * (Y.T @ Y) / s
    D = G - np.eye(n)
    t1 = r2 / s
    t2 = lam * float(np.sum(D * D)) / n ** 2
    dY1 = 2.0 * R / s - 2.0 * r2 * Y / s ** 2
    inner = float(np.sum(D * (Y.T @ Y)))
    dY2 = (lam / n ** 2) * ((4.0 * n / s) * (Y @ D) - (4.0 * n / s ** 2) * inner * Y)
    # coverage: 1 - tr(P Ge^-1 P^T) / nq with Ge = Y^T Y + eps I,
    # eps = delta s / n; with X = Ge^-1 P^T its gradient is
    # (mu / nq) (-2 Q X^T + 2 Y X X^T + (2 delta / n) ||X||^2 Y)
    eps = delta * s / n
    X = np.linalg.solve(Y.T @ Y + eps * np.eye(n), P.T)
    t3 = mu * (1.0 - float(np.trace(P @ X)) / nq)
    dY3 = (mu / nq) * (-2.0 * Q @ X.T + 2.0 * Y @ (X @ X.T) + (2.0 * delta / n) * float(np.sum(X * X)) * Y)
    return t1 + t2 + t3, dY1 + dY2 + dY3


def backward(params, cache, dY: np.ndarray):
    Fn, A1, A2 = cache
    g = {}
    g["W3"] = A2.T @ dY
    g["b3"] = dY.sum(axis=0)
    dA2 = dY @ params["W3"].T
    dZ2 = dA2 * (1.0 - A2 * A2)
    g["W2"] = A1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dA1 = dZ2 @ params["W2"].T
    dZ1 = dA1 * (1.0 - A1 * A1)
    g["W1"] = Fn.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


KEYS: List[str] = ["W1", "b1", "W2", "b2", "W3", "b3"]


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in KEYS:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[:] = b1 * m + (1 - b1) * grads[k]
        v[:] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + eps)
    return params


def flatten(params) -> np.ndarray:
    return np.concatenate([params[k].ravel() for k in KEYS])


def unflatten(vec: np.ndarray, din: int, hidden: int, dout: int):
    shapes = {"W1": (din, hidden), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,),
              "W3": (hidden, dout), "b3": (dout,)}
    out, o = {}, 0
    for k in KEYS:
        n = int(np.prod(shapes[k]))
        out[k] = vec[o:o + n].reshape(shapes[k]).copy()
        o += n
    return out
