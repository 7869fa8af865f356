"""Parity of chfsi_rayleigh_ritz_split (through the C ABI) with the oracle.

Tolerances.  FP64 mode: the Gram products sum M terms of size |x|^2
(relative rounding ~1e-15 after the chunked FP64 sums), and the Cholesky /
eigen solves of a well-conditioned random block (cond(S) < 1e3 here) lose
at most three more digits: eigenvalues at 1e-10 of max|theta|, vectors at
1e-9.  Mixed mode: the FP32 blocks carry relative errors of ~2^-24 sqrt(M)
in S and H^; the off-diagonal blocks are small on a nearly converged block,
so the top Ritz values (fr-fr block in FP64) stay within 1e-8 of the scale
and every value within 1e-5, as the oracle's own pins establish.
"""
import numpy as np
import pytest

import workloads
from oracle import density as dens
from oracle import fe
from oracle import rrgep

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2203_07820_amd as lib  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _sign_fix(A, R):
    s = np.sign(np.sum(A * R, axis=0))
    s[s == 0] = 1.0
    return A * s[None, :]


@pytest.mark.parametrize("case,N,nfr,pad", [
    ((3, 3, 2, 21), 24, 7, 0),
    ((2, 5, 2, 22), 150, 1, 5),      # two column tiles, ragged, ld > N
    ((3, 4, 2, 23), 200, 200, 0),     # every pair kept
    ((2, 6, 1, 24), 64, 16, 3),
])
def test_split_rr_fp64_matches_oracle(ctx, case, N, nfr, pad):
    nc, p, na, seed = case
    s = workloads.small_system(nc, p, na, seed=seed, has_proj=True)
    op = lib.Operator(ctx, s)
    ref_op = fe.build_operator(s)
    H = fe.assemble(ref_op)
    rng = np.random.default_rng(seed)
    Xh = rng.standard_normal((op.M, N + pad))
    X = torch.from_numpy(Xh).cuda()
    Pfr = torch.zeros(op.M, nfr + 2, dtype=torch.float64, device="cuda")
    th = op.rayleigh_ritz_split(X[:, :N] if pad else X, nfr, Pfr[:, :nfr])
    ref = rrgep.rrgep(lambda V: H @ V, Xh[:, :N], nfr)
    scale = np.max(np.abs(ref.theta))
    assert np.max(np.abs(th - ref.theta)) < 1e-10 * scale
    Xo = host(X)
    assert np.max(np.abs(Xo[:, :N] - ref.psi_o)) < 1e-9 * np.max(np.abs(ref.psi_o))
    if pad:
        assert np.array_equal(Xo[:, N:], Xh[:, N:])     # columns past N untouched
    got = _sign_fix(host(Pfr)[:, :nfr], ref.psi_fr)
    assert np.max(np.abs(got - ref.psi_fr)) < 1e-9 * np.max(np.abs(ref.psi_fr))
    assert np.all(host(Pfr)[:, nfr:] == 0.0)


@pytest.mark.parametrize("N,nfr", [(40, 8), (150, 20)])
def test_split_rr_mixed_precision_near_convergence(ctx, N, nfr):
    s = workloads.small_system(3, 5, 2, seed=13, has_proj=True)
    op = lib.Operator(ctx, s)
    ref_op = fe.build_operator(s)
    Hd = fe.dense(ref_op)
    lam, V = np.linalg.eigh(Hd)
    rng = np.random.default_rng(3)
    D = np.diag(rng.uniform(0.5, 2.0, N))
    Psi = (V[:, :N] + 1e-4 * rng.standard_normal((op.M, N))) @ D
    ref = rrgep.rrgep(lambda X: Hd @ X, Psi, nfr)
    X = torch.from_numpy(Psi.copy()).cuda()
    Pfr = torch.empty(op.M, nfr, dtype=torch.float64, device="cuda")
    th = op.rayleigh_ritz_split(X, nfr, Pfr, mixed=True)
    scale = np.max(np.abs(lam[:N]))
    assert np.max(np.abs(th[N - nfr:] - ref.theta[N - nfr:])) < 1e-8 * scale
    assert np.max(np.abs(th - ref.theta)) < 1e-5 * scale
    Xo = host(X)
    assert np.max(np.abs(Xo.T @ Xo - np.eye(N))) < 1e-5
    # the FP64 path on the same block is tight
    X2 = torch.from_numpy(Psi.copy()).cuda()
    th64 = op.rayleigh_ritz_split(X2, nfr, Pfr, mixed=False)
    assert np.max(np.abs(th64 - ref.theta)) < 1e-10 * scale


def test_split_rr_feeds_spectrum_split_density(ctx):
    # Algorithm 3 on the GPU path: rho(Psi_o, 2) + rho(Psi^R_fr, 2 (f - 1))
    # equals the oracle density of all Ritz vectors with weights 2 f
    s = workloads.small_system(3, 4, 2, seed=31, has_proj=True)
    op = lib.Operator(ctx, s)
    ref_op = fe.build_operator(s)
    H = fe.assemble(ref_op)
    N, nfr = 30, 6
    Xh = np.random.default_rng(7).standard_normal((op.M, N))
    X = torch.from_numpy(Xh.copy()).cuda()
    Pfr = torch.empty(op.M, nfr, dtype=torch.float64, device="cuda")
    th = op.rayleigh_ritz_split(X, nfr, Pfr)
    ne, kT = 2.0 * (N - nfr) + 3.0, 0.05
    mu, f = lib.fermi_level(th, ne, kT)
    f[:N - nfr] = 1.0                               # below the split: fully occupied
    rho = torch.zeros(op.M, dtype=torch.float64, device="cuda")
    op.density(X, np.full(N, 2.0), rho)
    op.density(Pfr, 2.0 * (f[N - nfr:] - 1.0), rho, accumulate=True)
    ref = rrgep.rrgep(lambda V: H @ V, Xh, nfr)
    full = dens.density(Xh @ ref.Q, 2.0 * f, ref_op.Mdiag)
    assert np.max(np.abs(host(rho) - full)) < 1e-9 * np.max(full)


@pytest.mark.parametrize("N,nfr,mixed", [(24, 5, False), (150, 12, False), (150, 12, True)])
def test_split_rr_complex_matches_oracle(ctx, N, nfr, mixed):
    s = workloads.small_system(2, 5, 2, seed=43, has_proj=True, k=(0.2, -0.1, 0.3))
    op = lib.Operator(ctx, s)
    ref_op = fe.build_operator(s)
    Hd = fe.dense(ref_op)
    lam, V = np.linalg.eigh(Hd)
    rng = np.random.default_rng(44)
    if mixed:   # nearly converged, unnormalised columns
        E = rng.standard_normal((op.M, N)) + 1j * rng.standard_normal((op.M, N))
        Psi = (V[:, :N] + 1e-4 * E) @ np.diag(rng.uniform(0.5, 2.0, N))
    else:
        Psi = rng.standard_normal((op.M, N)) + 1j * rng.standard_normal((op.M, N))
    ref = rrgep.rrgep(lambda X: Hd @ X, Psi, nfr)
    X = torch.from_numpy(Psi.copy()).cuda()
    Pfr = torch.zeros(op.M, nfr, dtype=torch.complex128, device="cuda")
    th = op.rayleigh_ritz_split(X, nfr, Pfr, mixed=mixed)
    scale = np.max(np.abs(ref.theta))
    Xo = host(X)
    if mixed:
        assert np.max(np.abs(th[N - nfr:] - ref.theta[N - nfr:])) < 1e-8 * scale
        assert np.max(np.abs(th - ref.theta)) < 1e-5 * scale
        assert np.max(np.abs(Xo.conj().T @ Xo - np.eye(N))) < 1e-5
    else:
        assert np.max(np.abs(th - ref.theta)) < 1e-10 * scale
        assert np.max(np.abs(Xo - ref.psi_o)) < 1e-9 * np.max(np.abs(ref.psi_o))
        # top Ritz vectors up to a phase per column
        got = host(Pfr)
        ph = np.sum(np.conj(got) * ref.psi_fr, axis=0)
        got = got * (ph / np.abs(ph))[None, :]
        assert np.max(np.abs(got - ref.psi_fr)) < 1e-9 * np.max(np.abs(ref.psi_fr))


def test_split_rr_rejects_bad_nfr(ctx):
    s2 = workloads.small_system(2, 3, 1, seed=42)
    op2 = lib.Operator(ctx, s2)
    X2 = torch.randn(op2.M, 8, dtype=torch.float64, device="cuda")
    P2 = torch.empty(op2.M, 9, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.ChfsiError):
        op2.rayleigh_ritz_split(X2, 9, P2)
