"""Parity of chfsi_density / chfsi_fermi_level (through the C ABI) with the
FP64 oracle.

Tolerance.  Every density value is a weighted sum of squares over ncols
columns (after at most 3 (p+1) multiply-adds of interpolation per value),
so FP64 rounding stays below (ncols + 3 (p+1)) * 2^-53 times the same sum
taken with |w_c| and |interpolated values|.  The tests allow 1e-12 of the
max of that absolute-weight density (ncols <= 1152 gives at most ~1.4e-13).
"""
import numpy as np
import pytest

import workloads
from oracle import density as dens
from oracle import fe

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


CASES = [
    # (ncell, p, natoms, k, seed)
    (2, 2, 1, (0, 0, 0), 11),
    (3, 3, 2, (0, 0, 0), 12),
    (2, 4, 2, (0.1, -0.2, 0.3), 13),
    (3, 5, 2, (0, 0, 0), 14),
    (2, 6, 2, (0.25, 0.0, -0.1), 15),
    (2, 7, 1, (0, 0, 0), 16),
]


def _block(op, ncols, ld, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((op.M, ld))
    if op.is_complex:
        X = X + 1j * rng.standard_normal((op.M, ld))
    return X


def _check(got, ref, scale):
    err = float(np.max(np.abs(got - ref)))
    assert err <= 1e-12 * float(np.max(scale)), (err, float(np.max(scale)))


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("ncols,pad", [(1, 0), (19, 3), (40, 0)])
def test_density_matches_oracle(ctx, case, ncols, pad):
    nc, p, na, k, seed = case
    s = workloads.small_system(nc, p, na, seed=seed, has_proj=True, k=k)
    op = lib.Operator(ctx, s)
    ld = ncols + pad
    Xh = _block(op, ncols, ld, seed + 100)
    w = np.random.default_rng(seed + 200).uniform(-1.0, 2.0, ncols)
    X = torch.from_numpy(Xh).cuda()
    Xv = X[:, :ncols] if pad else X
    Mdiag = fe.lumped_mass(nc, p, s.L)
    # nodes
    rho = torch.full((op.M,), 7.0, dtype=torch.float64, device="cuda")
    op.density(Xv, w, rho, points=lib.RHO_NODES)
    ref = dens.density(Xh[:, :ncols], w, Mdiag)
    _check(host(rho), ref, dens.density(Xh[:, :ncols], np.abs(w), Mdiag))
    # Gauss points of every cell
    rq = torch.full((op.E * (p + 1) ** 3,), 7.0, dtype=torch.float64, device="cuda")
    op.density(Xv, w, rq, points=lib.RHO_GAUSS)
    refq = dens.density_gauss(nc, p, s.L, Xh[:, :ncols], w).ravel()
    scale = dens.density_gauss(nc, p, s.L, np.abs(Xh[:, :ncols]), np.abs(w)).ravel()
    _check(host(rq), refq, scale)


@pytest.mark.parametrize("points", [0, 1])
def test_density_accumulates_split_blocks(ctx, points):
    # the spectrum-split form: rho from one call over all columns equals the
    # sum of two calls over column subsets (second call accumulates)
    s = workloads.small_system(3, 4, 2, seed=21, has_proj=True)
    op = lib.Operator(ctx, s)
    Xh = _block(op, 48, 48, 22)
    w = np.random.default_rng(23).uniform(-0.5, 2.0, 48)
    n_out = op.M if points == 0 else op.E * 125
    r1 = torch.zeros(n_out, dtype=torch.float64, device="cuda")
    r2 = torch.zeros_like(r1)
    X = torch.from_numpy(Xh).cuda()
    op.density(X, w, r1, points=points)
    A = X[:, :30].contiguous()
    B = X[:, 30:].contiguous()
    op.density(A, w[:30], r2, points=points)
    op.density(B, w[30:], r2, points=points, accumulate=True)
    a, b = host(r1), host(r2)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_density_of_ground_state_integrates_to_electron_count(ctx):
    # end to end on the GPU path: Ritz pairs from the solver, mu and f from
    # chfsi_fermi_level, rho from chfsi_density; the lumped quadrature of the
    # nodal density returns N_e (Ritz vectors are M-orthonormal)
    s = workloads.small_system(3, 4, 2, seed=31, has_proj=True)
    op = lib.Operator(ctx, s)
    N, nb = 24, 8
    X = torch.from_numpy(workloads.start_block(op.M, N + nb, seed=32)).cuda()
    theta, resid, _ = op.solve(X, nwanted=N, n_buf=nb, m=20, block=N + nb, tol=1e-9, max_passes=60)
    ne, kT = 30.0, 0.01
    mu, f = lib.fermi_level(theta[:N], ne, kT)
    rho = torch.zeros(op.M, dtype=torch.float64, device="cuda")
    op.density(X[:, :N].contiguous(), 2.0 * f, rho)
    Mdiag = fe.lumped_mass(3, 4, s.L)
    assert abs(float(np.sum(host(rho) * Mdiag)) - ne) < 1e-8


def test_fermi_level_matches_oracle():
    rng = np.random.default_rng(41)
    th = np.sort(rng.uniform(-2.0, 1.0, 200))
    for ne, kT, w in ((150.0, 0.003, None), (37.5, 0.05, None), (80.0, 0.01, rng.uniform(0.1, 1.0, 200))):
        mu, occ = lib.fermi_level(th, ne, kT, weights=w)
        mu_ref = dens.fermi_level(th, ne, kT, weights=w)
        assert abs(mu - mu_ref) < 1e-12
        assert np.max(np.abs(occ - dens.occupations(th, mu_ref, kT))) < 1e-10
    with pytest.raises(lib.ChfsiError):
        lib.fermi_level(th, 400.0, 0.01)   # more electrons than states


def test_density_c2_block_sampled(ctx):
    # the full c1 operator (24^3 cells, p = 6, M = 2,985,984) with the c2 block
    # width (1024 + 128 columns) that bench.py times; sampled nodes and cells
    # against the oracle
    s = workloads.config("c1")
    op = lib.Operator(ctx, s)
    ncols = 1152
    g = torch.Generator(device="cuda").manual_seed(51)
    X = torch.randn(op.M, ncols, dtype=torch.float64, device="cuda", generator=g)
    w = np.random.default_rng(52).uniform(0.0, 2.0, ncols)
    rho = torch.empty(op.M, dtype=torch.float64, device="cuda")
    rq = torch.empty(op.E * 343, dtype=torch.float64, device="cuda")
    op.density(X, w, rho, points=lib.RHO_NODES)
    op.density(X, w, rq, points=lib.RHO_GAUSS)
    torch.cuda.synchronize()
    rng = np.random.default_rng(53)
    Mdiag = fe.lumped_mass(s.ncell, s.p, s.L)
    rows = np.concatenate([[0, op.M - 1], rng.integers(0, op.M, 2000)])
    Xr = X[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = dens.density(Xr, w, Mdiag[rows])
    got = rho.cpu().numpy()[rows]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(ref)
    cells = np.concatenate([[0, op.E - 1], rng.integers(0, op.E, 40)])
    nodes = fe.cell_nodes(s.ncell, s.p)[cells]
    uniq, inv = np.unique(nodes.ravel(), return_inverse=True)
    Xu = X[torch.from_numpy(uniq).cuda()].cpu().numpy()
    D = 1.0 / np.sqrt(Mdiag[uniq])
    Ph = (D[:, None] * Xu)[inv.reshape(nodes.shape)]
    gotq = rq.view(op.E, 343).cpu().numpy()[cells]
    for i in range(cells.size):
        refq = dens.density_gauss_cell(s.p, Ph[i], w)
        scale = dens.density_gauss_cell(s.p, np.abs(Ph[i]), w)
        assert np.max(np.abs(gotq[i] - refq)) <= 1e-12 * np.max(scale)
