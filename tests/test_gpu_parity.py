"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances.  FP64 paths: the cell products sum at most 8 * mcell terms of
size |A| |X| per entry, so rounding stays below 1e-13 of max|Y|; the tests
use 1e-12 relative to the max-norm.  Single-precision paths: unit roundoff
6e-8 times the same growth, tested at 2e-5 relative.  Eigenvalues after
the same number of passes: 1e-8 Ha (FP64).
"""
import math

import numpy as np
import scipy.sparse.linalg as spla
import pytest

import workloads
from oracle import chfsi as ochfsi
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


SMALL = [
    # (ncell, p, natoms, proj, k, seed)
    (2, 2, 1, False, (0, 0, 0), 1),
    (3, 3, 2, True, (0, 0, 0), 2),
    (2, 4, 2, True, (0, 0, 0), 3),
    (3, 5, 3, True, (0, 0, 0), 4),
    (2, 6, 2, True, (0, 0, 0), 5),
    (3, 4, 2, True, (0.1, -0.2, 0.3), 6),
    (2, 5, 2, True, (0.25, 0.0, -0.1), 7),
    (2, 7, 1, True, (0, 0, 0), 8),
]


def _sys(nc, p, na, proj, k, seed, L=None):
    return workloads.small_system(nc, p, na, seed=seed, has_proj=proj, k=k, L=L)


@pytest.mark.parametrize("case", SMALL)
def test_operator_tables_match_oracle(ctx, case):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    ref = fe.build_operator(s)
    t = op.tables()
    assert op.M == ref.M and op.E == ref.E
    assert np.max(np.abs(t["xyz"] - fe.node_coords(s.ncell, s.p, s.L))) < 1e-13
    assert relerr(t["dscale"], ref.D) < 1e-14
    assert np.max(np.abs(t["vdiag"] - (ref.V + 0.5 * ref.k @ ref.k))) < 1e-13
    # the GPU's shared cell matrix is D_c (K^c/2 - i skew(k.G^c)/2) D_c
    Dc = ref.D[ref.cells[0]]
    Ge = np.einsum("a,aij->ij", ref.k, ref.ct.G)
    A = Dc[:, None] * (0.5 * ref.ct.K - 0.5j * (Ge - Ge.T)) * Dc[None, :]
    if not op.is_complex:
        A = A.real
    assert relerr(t["cell"], A) < 1e-13


@pytest.mark.parametrize("case", SMALL)
@pytest.mark.parametrize("ncols", [1, 37, 64, 130])
def test_apply_fp64_matches_oracle(ctx, case, ncols):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    if ncols > op.M:
        pytest.skip("more columns than nodes is rejected by design")
    ref = fe.build_operator(s)
    H = fe.assemble(ref)
    X = workloads.start_block(op.M, ncols, seed=100 + ncols, complex_=op.is_complex)
    Y = np.zeros_like(X)
    Xd, Yd = dev(X), dev(Y)
    op.apply(Xd, Yd)
    Yg = host(Yd)
    assert relerr(Yg, H @ X) < 1e-12


@pytest.mark.parametrize("case", [SMALL[2], SMALL[4], SMALL[5]])
def test_apply_with_leading_dimension(ctx, case):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    X = workloads.start_block(op.M, 50, seed=3, complex_=op.is_complex)
    Xd = dev(X)
    Yd = torch.zeros_like(Xd)
    # the first 20 columns of the 50-wide buffers, passed as (ncols, ld)
    ncols, ld = 20, 50
    op.ctx.check(op.ctx.lib.chfsi_apply(op.h, lib._tptr(Xd), lib._tptr(Yd), ncols, ld,
                                        lib.C128 if op.is_complex else lib.F64))
    Yg = host(Yd)
    assert relerr(Yg[:, :20], H @ X[:, :20]) < 1e-12
    assert np.all(Yg[:, 20:] == 0)


# every order: real FP32 takes four column tiles per wave for p <= 6 and two
# at p = 7; complex FP32 two
@pytest.mark.parametrize("case", SMALL)
def test_apply_fp32_matches_oracle(ctx, case):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    X = workloads.start_block(op.M, min(70, op.M - 4), seed=11, complex_=op.is_complex)
    dt = np.complex64 if op.is_complex else np.float32
    Xd = dev(X.astype(dt))
    Yd = torch.zeros_like(Xd)
    op.apply(Xd, Yd, lib.C64 if op.is_complex else lib.F32)
    Yg = host(Yd).astype(np.complex128 if op.is_complex else np.float64)
    ref = H @ X.astype(dt).astype(X.dtype)
    assert relerr(Yg, ref) < 2e-5


@pytest.mark.parametrize("case", [SMALL[1], SMALL[3], SMALL[5]])
def test_filter_fp64_matches_oracle(ctx, case):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    lam = np.linalg.eigvalsh(H.toarray())
    X = workloads.start_block(op.M, 24, seed=5, complex_=op.is_complex)
    a, b, aL = lam[24], lam[-1] * 1.05, lam[0]
    Yref = ochfsi.cheb_filter(lambda v: H @ v, X, 12, a, b, aL)
    Xd = dev(X)
    op.filter(Xd, 12, a, b, aL, block=10)
    assert relerr(host(Xd), Yref) < 1e-11


def test_filter_fp32_close_to_oracle(ctx):
    s = _sys(*SMALL[3])
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    lam = np.linalg.eigvalsh(H.toarray())
    X = workloads.start_block(op.M, 16, seed=6)
    a, b, aL = lam[16], lam[-1] * 1.05, lam[0]
    Yref = ochfsi.cheb_filter(lambda v: H @ v, X, 10, a, b, aL)
    Xd = dev(X)
    op.filter(Xd, 10, a, b, aL, prec=lib.F32)
    assert relerr(host(Xd), Yref) < 1e-4


@pytest.mark.parametrize("case", [SMALL[2], SMALL[5]])
def test_orthonormalize_matches_oracle(ctx, case):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    X = workloads.start_block(op.M, 40, seed=8, complex_=op.is_complex)
    Xo, Lref, _ = ochfsi.cholgs(X)
    Xd = dev(X)
    L = op.orthonormalize(Xd, want_L=True)
    assert relerr(host(Xd), Xo) < 1e-12
    assert relerr(L, Lref) < 1e-12


@pytest.mark.parametrize("k", [(0, 0, 0), (0.1, -0.2, 0.15)])
def test_subspace_kernels_multi_tile(ctx, k):
    # 200 columns (400 in the real view of a complex block): several
    # 128-wide Gram tiles, two or more rotation column blocks, the triangular
    # cut-off of X L^-H, and an odd row count (15^3 = 3375) that leaves a
    # ragged last k step
    s = workloads.small_system(3, 5, 2, seed=21, has_proj=True, k=k)
    op = lib.Operator(ctx, s)
    N = 200
    X = workloads.start_block(op.M, N, seed=22, complex_=op.is_complex)
    Xo, Lref, _ = ochfsi.cholgs(X)
    Xd = dev(X)
    L = op.orthonormalize(Xd, want_L=True)
    assert relerr(host(Xd), Xo) < 1e-11
    assert relerr(L, Lref) < 1e-11
    H = fe.assemble(fe.build_operator(s))
    th_ref, Psi_ref, _, r_ref, _ = ochfsi.rayleigh_ritz(lambda v: H @ v, Xo)
    th, r = op.rayleigh_ritz(Xd)
    assert np.max(np.abs(th - th_ref)) < 1e-10 * max(1.0, np.max(np.abs(th_ref)))
    assert np.max(np.abs(r - r_ref)) < 1e-9


def test_orthonormalize_with_trailing_gram_chunks(ctx):
    # M = 45^3 = 91,125 rows and 200 columns: 342 row chunks of 272 rows
    # would cover more than M, so the launch must not leave chunks (and their
    # partial tiles) empty
    s = workloads.small_system(15, 3, 2, seed=23)
    op = lib.Operator(ctx, s)
    X = workloads.start_block(op.M, 200, seed=24)
    Xo, Lref, _ = ochfsi.cholgs(X)
    Xd = dev(X)
    L = op.orthonormalize(Xd, want_L=True)
    assert relerr(L, Lref) < 1e-11
    assert relerr(host(Xd), Xo) < 1e-10


def test_orthonormalize_rank_deficient_fails(ctx):
    s = _sys(*SMALL[1])
    op = lib.Operator(ctx, s)
    X = workloads.start_block(op.M, 10, seed=9)
    X[:, 4] = X[:, 2]
    Xd = dev(X)
    with pytest.raises(lib.ChfsiError) as ei:
        op.orthonormalize(Xd)
    assert ei.value.code == -4
    assert np.array_equal(host(Xd), X)


# Blocks of at most 64 columns take the one-workgroup Cholesky-inverse and
# Jacobi eigensolver kernels; 65 columns the library route beside them.
@pytest.mark.parametrize("N", [1, 2, 17, 64, 65])
@pytest.mark.parametrize("case", [SMALL[2], SMALL[5]])
def test_small_block_orthonormalize_and_rayleigh_ritz(ctx, case, N):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    X = workloads.start_block(op.M, N, seed=31 + N, complex_=op.is_complex)
    Xo, _, _ = ochfsi.cholgs(X)
    Xd = dev(X)
    op.orthonormalize(Xd)             # no factor requested: the small kernel for N <= 64
    assert relerr(host(Xd), Xo) < 1e-12
    H = fe.assemble(fe.build_operator(s))
    th_ref, Psi_ref, _, r_ref, _ = ochfsi.rayleigh_ritz(lambda v: H @ v, Xo)
    th, r = op.rayleigh_ritz(Xd)
    assert np.all(np.diff(th) >= 0)
    assert np.max(np.abs(th - th_ref)) < 1e-11 * max(1.0, np.max(np.abs(th_ref)))
    assert np.max(np.abs(r - r_ref)) < 1e-10
    Psi = host(Xd)
    # Ritz vectors orthonormal and spanning the oracle's Ritz vectors (per
    # column up to a unit phase where the Ritz values are distinct)
    assert np.max(np.abs(Psi.conj().T @ Psi - np.eye(N))) < 1e-12
    ph = np.sum(Psi.conj() * Psi_ref, axis=0)
    ph = ph / np.abs(ph)
    assert relerr(Psi * ph[None, :], Psi_ref) < 1e-9


def test_small_block_rayleigh_ritz_degenerate(ctx):
    # free electrons (V = 0, k = 0): the 6-fold |n|^2 = 1 shell makes the
    # projected matrix of a block that holds it exactly degenerate; compare
    # eigenvalues and the projector onto each cluster, not the vectors
    s = workloads.small_system(2, 4, 0, seed=41)
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    lam, Q = np.linalg.eigh(H.toarray())
    N = 20
    rng = np.random.default_rng(42)
    X = Q[:, :N] @ np.linalg.qr(rng.standard_normal((N, N)))[0]   # the lowest 20 states, rotated
    Xd = dev(X)
    th, r = op.rayleigh_ritz(Xd)
    assert np.max(np.abs(th - lam[:N])) < 1e-11 * max(1.0, np.max(np.abs(lam[:N])))
    assert np.max(r) < 1e-10
    Psi = host(Xd)
    cuts = np.nonzero(np.diff(lam[:N + 1]) > 1e-8)[0] + 1
    lo = 0
    for hi in cuts:
        P = Psi[:, lo:hi] @ Psi[:, lo:hi].T
        Pr = Q[:, lo:hi] @ Q[:, lo:hi].T
        assert np.max(np.abs(P - Pr)) < 1e-10
        lo = hi


@pytest.mark.parametrize("case", [SMALL[2], SMALL[5]])
def test_rayleigh_ritz_matches_oracle(ctx, case):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    X = workloads.start_block(op.M, 30, seed=10, complex_=op.is_complex)
    Xo, _, _ = ochfsi.cholgs(X)
    th_ref, Psi_ref, _, r_ref, _ = ochfsi.rayleigh_ritz(lambda v: H @ v, Xo)
    Xd = dev(Xo)
    th, r = op.rayleigh_ritz(Xd)
    assert np.max(np.abs(th - th_ref)) < 1e-11 * max(1.0, np.max(np.abs(th_ref)))
    assert np.max(np.abs(r - r_ref)) < 1e-10
    Psi = host(Xd)
    # vectors are unique up to a unit phase per column (distinct Ritz values)
    ph = np.sum(Psi.conj() * Psi_ref, axis=0)
    ph = ph / np.abs(ph)
    assert relerr(Psi * ph[None, :], Psi_ref) < 1e-9


@pytest.mark.parametrize("case", [SMALL[2], SMALL[5]])
def test_bounds_match_oracle(ctx, case):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    v0 = workloads.lanczos_start(op.M, seed=44, complex_=op.is_complex)
    b_ref, tmin, _, _ = ochfsi.lanczos_bound(lambda v: H @ v, v0, 20)
    b, lmin = op.bounds(20, dev(v0))
    assert abs(b - b_ref) < 1e-9 * abs(b_ref)
    assert abs(lmin - tmin) < 1e-9 * max(1.0, abs(tmin))
    assert b >= np.linalg.eigvalsh(H.toarray())[-1]


def test_solve_config0_matches_oracle_pass_by_pass(ctx):
    s = workloads.config("c0")
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    N = 32
    X0 = workloads.start_block(op.M, N, seed=s.seed + 1_000_000)
    v0 = workloads.lanczos_start(op.M, seed=s.seed + 2_000_000)
    ref = ochfsi.solve(lambda v: H @ v, X0, N, m=20, block=32, v0=v0, passes=10)
    Xd = dev(X0)
    th, r, st = op.solve(Xd, N, m=20, block=32, fixed_passes=10, lanczos_v0=v0)
    assert st["passes"] == 10
    assert abs(st["b_upper"] - ref.b) < 1e-9 * ref.b
    assert np.max(np.abs(th - ref.theta)) < 1e-8
    lam = np.linalg.eigvalsh(H.toarray())
    assert np.max(np.abs(th[:28] - lam[:28])) < 1e-8
    Psi = host(Xd)
    assert np.max(np.abs(Psi.T @ Psi - np.eye(N))) < 1e-12


def test_error_paths(ctx):
    s = _sys(*SMALL[1])
    op = lib.Operator(ctx, s)
    X = dev(np.zeros((op.M, 4)))
    Y = dev(np.zeros((op.M, 4)))
    with pytest.raises(lib.ChfsiError):   # precision does not match a real operator
        op.apply(X, Y, lib.C128)
    with pytest.raises(lib.ChfsiError):   # aL >= a
        op.filter(X, 5, 1.0, 2.0, 1.5)
    with pytest.raises(lib.ChfsiError):   # a >= b
        op.filter(X, 5, 3.0, 2.0, 0.0)
    with pytest.raises(lib.ChfsiError):   # X == Y
        op.apply(X, X)
    bad = workloads.small_system(2, 9, 1, seed=1)
    with pytest.raises(lib.ChfsiError):   # order outside [2, 7]
        lib.Operator(ctx, bad)


REAL = [c for c in SMALL if not any(c[4])]


@pytest.mark.parametrize("case", REAL)
def test_apply_bf16_matches_oracle_rounded_scheme(ctx, case):
    # BF16 scheme: cell products on bf16-rounded inputs with FP32 accumulation;
    # the oracle forms the same rounded inputs and sums in FP64, so only the
    # FP32 accumulation differs (tolerance 2e-5 of max|Y|).
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    ref_op = fe.build_operator(s)
    X = workloads.start_block(op.M, min(70, op.M), seed=12).astype(np.float32)
    Xd = dev(X)
    Yd = torch.zeros_like(Xd)
    op.apply(Xd, Yd, lib.BF16)
    Yg = host(Yd).astype(np.float64)
    ref = fe.apply_cellwise_bf16(ref_op, X.astype(np.float64))
    assert relerr(Yg, ref) < 2e-5
    # and the rounding is visible: the bf16 result differs from the FP64 one
    H = fe.assemble(ref_op)
    assert relerr(Yg, H @ X.astype(np.float64)) > 1e-4


@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("case", REAL)
def test_filter_bf16_matches_oracle_rounded_scheme(ctx, case, m):
    # the fused recurrence steps of the BF16 filter (owner's diagonal term,
    # -beta X_{k-1}, clearing of X_{k-1}) against the oracle's filter with the
    # same bf16-rounded cell products.  One step (m = 1) rounds only the
    # input block, which both sides hold exactly: FP32 accumulation sets the
    # tolerance.  From the second step on, each side rounds its own iterate
    # to bf16 (the kernel's FP32 iterate, the oracle's FP64 one); where they
    # straddle a rounding boundary the products differ by a bf16 ulp of that
    # entry times a cell-matrix column, so the check is on the Frobenius norm
    # (a perturbation of 2e-6 of the iterates moves it by at most 4e-4 on
    # these systems) and loosely on the maximum; a missing or doubled
    # -beta X_{k-1} term or an uncleared target would be O(1) in both.
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    ref_op = fe.build_operator(s)
    H = fe.assemble(ref_op)
    lmax = float(spla.eigsh(H, k=1, which="LA", return_eigenvectors=False)[0])
    a, b, aL = 0.05 * lmax, 1.05 * lmax, -0.1 * lmax
    X = workloads.start_block(op.M, min(70, op.M), seed=13).astype(np.float32)
    ref = ochfsi.cheb_filter(lambda v: fe.apply_cellwise_bf16(ref_op, v), X.astype(np.float64), m, a, b, aL)
    Xd = dev(X.astype(np.float64))
    op.filter(Xd, m, a, b, aL, prec=lib.BF16)
    got = host(Xd)
    if m == 1:
        assert relerr(got, ref) < 5e-5
    else:
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 2e-3
        assert relerr(got, ref) < 3e-2


def test_filter_bf16_close_to_oracle(ctx):
    s = _sys(*SMALL[3])
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    lam = np.linalg.eigvalsh(H.toarray())
    X = workloads.start_block(op.M, 16, seed=6)
    a, b, aL = lam[16], lam[-1] * 1.05, lam[0]
    Yref = ochfsi.cheb_filter(lambda v: H @ v, X, 10, a, b, aL)
    Xd = dev(X)
    op.filter(Xd, 10, a, b, aL, prec=lib.BF16)
    # the filtered block keeps its direction to bf16 accuracy
    assert relerr(host(Xd), Yref) < 3e-2
