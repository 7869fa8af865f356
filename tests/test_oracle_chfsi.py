"""Pins of the oracle's ChFSI iteration: the explicit Chebyshev polynomial,
dense LAPACK eigendecompositions, orthonormality, interlacing, the Lanczos
bound.  Every reference value here comes from a route other than the
oracle's own recurrence or Rayleigh-Ritz code."""
import numpy as np
import pytest

import workloads
from oracle import chfsi, fe


def _rand_sym(n, seed, complex_=False):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    if complex_:
        A = A + 1j * rng.standard_normal((n, n))
    return 0.5 * (A + A.conj().T)


@pytest.mark.parametrize("complex_", [False, True])
def test_P5_scaled_recurrence_equals_explicit_polynomial(complex_):
    n, m = 60, 20
    H = _rand_sym(n, 1, complex_)
    lam, Q = np.linalg.eigh(H)
    a, b, aL = lam[15], lam[-1] + 0.1, lam[0]
    X = workloads.start_block(n, 7, seed=3, complex_=complex_)
    Y = chfsi.cheb_filter(lambda v: H @ v, X, m, a, b, aL)
    f = chfsi.cheb_explicit(lam, m, a, b, aL)
    Yref = Q @ (f[:, None] * (Q.conj().T @ X))
    assert np.max(np.abs(Y - Yref)) <= 1e-12 * np.max(np.abs(Yref))


def test_explicit_chebyshev_matches_numpy_chebyshev_series():
    # T_m from the closed form equals numpy's Chebyshev series evaluation.
    t = np.linspace(-3, 3, 41)
    m = 9
    ref = np.polynomial.chebyshev.chebval(t, [0] * m + [1])
    got = chfsi.cheb_explicit(t, m, -1.0, 1.0, -2.0) * np.polynomial.chebyshev.chebval(-2.0, [0] * m + [1])
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_filter_rejects_bad_interval():
    with pytest.raises(ValueError):
        chfsi.cheb_filter(lambda v: v, np.ones((3, 1)), 4, 1.0, 0.5, 0.0)


def test_P10_lanczos_bound_above_spectrum():
    s = workloads.small_system(2, 4, 2, seed=21, has_proj=True)
    op = fe.build_operator(s)
    H = fe.assemble(op)
    lmax = np.linalg.eigvalsh(H.toarray())[-1]
    for seed in range(5):
        v0 = workloads.lanczos_start(op.M, seed)
        b, tmin, tmax, fn = chfsi.lanczos_bound(lambda v: H @ v, v0, 20)
        assert b >= lmax
        assert tmax <= lmax + 1e-10
        assert b < 2.0 * lmax


def test_P6_cholgs_orthonormal_and_same_span():
    X = workloads.start_block(500, 24, seed=5, complex_=True)
    Xo, L, S = chfsi.cholgs(X)
    assert np.max(np.abs(Xo.conj().T @ Xo - np.eye(24))) < 1e-12
    assert np.allclose(Xo @ L.conj().T, X, atol=1e-12)
    with pytest.raises(np.linalg.LinAlgError):
        Y = X.copy()
        Y[:, 3] = Y[:, 7]
        chfsi.cholgs(Y)


def test_rayleigh_ritz_exact_on_invariant_subspace():
    H = _rand_sym(80, 2)
    lam, Q = np.linalg.eigh(H)
    R = np.linalg.qr(np.random.default_rng(0).standard_normal((10, 10)))[0]
    Xo = Q[:, 5:15] @ R
    th, Psi, HPsi, r, _ = chfsi.rayleigh_ritz(lambda v: H @ v, Xo)
    assert np.max(np.abs(th - lam[5:15])) < 1e-12
    assert np.max(r) < 1e-12
    assert np.max(np.abs(Psi.T @ Psi - np.eye(10))) < 1e-12


def test_P4_P9_config0_converges_to_dense_eigenvalues():
    # The first workload: L = 10, 4^3 cells, p = 4, two Gaussian atoms,
    # N = 32, m = 20, random start, passes of filter + CholGS + RR.
    s = workloads.config("c0")
    op = fe.build_operator(s)
    H = fe.assemble(op)
    lam = np.linalg.eigvalsh(H.toarray())
    N = 32
    X0 = workloads.start_block(op.M, N, seed=s.seed + 1_000_000)
    v0 = workloads.lanczos_start(op.M, seed=s.seed + 2_000_000)
    res = chfsi.solve(lambda v: H @ v, X0, N, m=20, block=32, v0=v0, passes=10)
    assert res.b >= lam[-1]
    # Cauchy interlacing (theta_i >= lambda_i) and monotone decrease per pass
    for th in res.history:
        assert np.all(th - lam[:N] >= -1e-12)
    for t0, t1 in zip(res.history[1:], res.history[2:]):
        assert np.all(t1 <= t0 + 1e-12)
    # converged to dense eigenvalues within 1e-8 Ha for the states below the
    # top few (the last wanted state converges slowest: index 32 sits in a
    # cluster)
    assert np.max(np.abs(res.theta[:28] - lam[:28])) < 1e-8
    assert np.max(np.abs(res.X.T @ res.X - np.eye(N))) < 1e-12
    # with 8 buffer columns (the filter damps everything above the largest
    # Ritz value, so the last wanted state needs a gap) every wanted pair
    # reaches a tight residual and matches dense eigh
    Xb = np.concatenate([res.X, workloads.start_block(op.M, 8, seed=77)], axis=1)
    res2 = chfsi.solve(lambda v: H @ v, Xb, N, m=20, block=40, v0=v0, tol=1e-9,
                       max_passes=60, b=res.b)
    assert np.max(res2.resid) <= 1e-9
    assert np.max(np.abs(res2.theta - lam[:N])) < 1e-10
