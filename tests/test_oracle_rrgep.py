"""Pins of the spectrum-splitting Rayleigh-Ritz oracle (no GPU).

* Invariant subspace: for Psi_f = V R (V the exact lowest N eigenvectors of
  a small operator, R a random non-orthogonal mixing), the generalised
  eigenvalues are the exact eigenvalues, Psi_o is orthonormal with the span
  of V, and Psi^R_fr spans the N_fr highest of them.
* The generalised route equals the orthonormalise-then-project route
  (Cholesky-Gram-Schmidt, then Rayleigh-Ritz) of the other oracle module on
  a random block: same Ritz values and the same orthonormal basis.
* Mixed precision on a nearly converged block stays within the FP32 error
  of the FP64 result, while a plain FP32 evaluation of everything is pinned
  to be visibly worse on the top Ritz values (the FP64 parts matter).
* Spectrum-split density: rho(Psi_o, 2) + rho(Psi^R_fr, 2 (f - 1)) equals the
  density of all Ritz vectors with weights 2 f (f = 1 below the split).
"""
import numpy as np

import workloads
from oracle import chfsi as ochfsi
from oracle import density as dens
from oracle import fe
from oracle import rrgep


def _setup(nc=3, p=4, na=2, seed=9, k=(0.0, 0.0, 0.0)):
    s = workloads.small_system(nc, p, na, seed=seed, has_proj=True, k=k)
    op = fe.build_operator(s)
    H = fe.dense(op)
    lam, V = np.linalg.eigh(H)
    return op, H, lam, V


def test_invariant_subspace_gives_exact_pairs():
    for k in ((0.0, 0.0, 0.0), (0.2, -0.1, 0.3)):
        op, H, lam, V = _setup(k=k)
        N, nfr = 20, 6
        rng = np.random.default_rng(1)
        R = np.triu(rng.standard_normal((N, N))) + 3.0 * np.eye(N)
        if np.iscomplexobj(V):
            R = R + 0.3j * np.triu(rng.standard_normal((N, N)), 1)
        Psi = V[:, :N] @ R
        r = rrgep.rrgep(lambda X: H @ X, Psi, nfr)
        assert np.max(np.abs(r.theta - lam[:N])) < 1e-10 * np.max(np.abs(lam[:N]))
        assert np.max(np.abs(r.psi_o.conj().T @ r.psi_o - np.eye(N))) < 1e-12
        Pv = V[:, :N] @ V[:, :N].conj().T
        assert np.max(np.abs(Pv @ r.psi_o - r.psi_o)) < 1e-11
        # top N_fr Ritz vectors: the projector onto them equals the exact one
        # (lam[N-nfr-1] < lam[N-nfr], a gap, for this operator)
        Ptop = V[:, N - nfr:N] @ V[:, N - nfr:N].conj().T
        Pfr = r.psi_fr @ r.psi_fr.conj().T
        assert lam[N - nfr] - lam[N - nfr - 1] > 1e-3
        assert np.max(np.abs(Pfr - Ptop)) < 1e-9


def test_generalised_route_equals_orthonormalise_then_project():
    op, H, lam, V = _setup(seed=11)
    rng = np.random.default_rng(2)
    Psi = rng.standard_normal((op.M, 24))
    r = rrgep.rrgep(lambda X: H @ X, Psi, 24)
    Xo, _, _ = ochfsi.cholgs(Psi)
    th_rr = ochfsi.rayleigh_ritz(lambda X: H @ X, Xo)[0]
    assert np.max(np.abs(r.theta - th_rr)) < 1e-9 * np.max(np.abs(th_rr))
    # the two orthonormal bases are the same matrix (same Cholesky factor)
    assert np.max(np.abs(r.psi_o - Xo)) < 1e-10


def test_mixed_precision_error_is_fp32_sized_and_fp64_parts_matter():
    op, H, lam, V = _setup(nc=3, p=5, seed=13)
    N, nfr = 40, 8
    rng = np.random.default_rng(3)
    D = np.diag(rng.uniform(0.5, 2.0, N))           # unnormalised columns
    Psi = (V[:, :N] + 1e-4 * rng.standard_normal((op.M, N))) @ D
    ref = rrgep.rrgep(lambda X: H @ X, Psi, nfr)
    mix = rrgep.rrgep(lambda X: H @ X, Psi, nfr, mixed=True, block=16)
    scale = np.max(np.abs(lam[:N]))
    err_mix = np.max(np.abs(mix.theta[N - nfr:] - ref.theta[N - nfr:]))
    assert err_mix < 1e-8 * scale      # the fr-fr block in FP64 carries the top pairs
    assert np.max(np.abs(mix.psi_o.T @ mix.psi_o - np.eye(N))) < 1e-5
    # everything in FP32 (no FP64 blocks at all): much larger top-pair error
    P32 = Psi.astype(np.float32)
    S = (P32.T @ P32).astype(np.float64)
    Hh = (P32.T @ (H @ Psi).astype(np.float32)).astype(np.float64)
    L = np.linalg.cholesky(0.5 * (S + S.T))
    Li = np.linalg.inv(L)
    th32 = np.linalg.eigvalsh(0.5 * (Li @ Hh @ Li.T + (Li @ Hh @ Li.T).T))
    assert np.max(np.abs(th32[N - nfr:] - ref.theta[N - nfr:])) > 100.0 * err_mix


def test_spectrum_split_density_identity():
    op, H, lam, V = _setup(seed=17)
    N, nfr = 18, 5
    rng = np.random.default_rng(5)
    Psi = rng.standard_normal((op.M, N))
    r = rrgep.rrgep(lambda X: H @ X, Psi, nfr)
    f = np.ones(N)
    f[N - nfr:] = (0.9, 0.6, 0.3, 0.1, 0.02)
    ritz = Psi @ r.Q
    full = dens.density(ritz, 2.0 * f, op.Mdiag)
    split = dens.density(r.psi_o, np.full(N, 2.0), op.Mdiag) \
        + dens.density(r.psi_fr, 2.0 * (f[N - nfr:] - 1.0), op.Mdiag)
    assert np.max(np.abs(full - split)) < 1e-11 * np.max(full)
