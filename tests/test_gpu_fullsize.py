"""Full-size parity: the production operators in the launch configuration the
benchmark times (one 128-column block per launch), checked on sampled rows
that the oracle computes one by one from the cells containing them.

* c1 (24^3 cells, p = 6, M = 2,985,984, 64 atoms with projectors): H~X and
  one fused filter step (m = 1, alpha (H~X - cX)) in FP64 and FP32, and H~X
  in the BF16 scheme against the oracle's identically rounded products.
* the largest c3 operator (20^3 cells, p = 5) at its first k-point, complex128
  and complex64.
* c1 with the per-cell Gauss-quadrature potential: H~X.

Tolerances as in the small-size parity tests: FP64 1e-12 and FP32 2e-5
relative to the largest sampled magnitude.
"""
import numpy as np
import pytest

import workloads
from oracle import chfsi as ochfsi
from oracle import dhm
from oracle import fe

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2203_07820_amd as lib  # noqa: E402

B = 128


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def _rows(M, n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, M - 1], rng.integers(0, M, n)]))


def _block(M, cplx, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    if cplx:
        return torch.randn(M, B, dtype=torch.complex128, device="cuda", generator=g)
    return torch.randn(M, B, dtype=torch.float64, device="cuda", generator=g)


def _gather_rows(X, rows):
    return X[torch.from_numpy(rows).cuda()].cpu().numpy()


def test_c1_apply_and_filter_step_sampled(ctx):
    s = workloads.config("c1")
    op = lib.Operator(ctx, s)
    ref = fe.build_operator(s)
    X = _block(op.M, False, 101)
    Y = torch.zeros_like(X)
    op.apply(X, Y)
    rows = _rows(op.M, 60, 102)
    Xh = X.cpu().numpy()
    want = fe.apply_rows(ref, Xh, rows)
    got = _gather_rows(Y, rows)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    # one fused recurrence step of the filter, F64 and F32
    b, _ = op.bounds(20, seed=1)
    a, aL = 0.1 * b, -1.0
    c, co = ochfsi.cheb_coeffs(1, a, b, aL)
    step = co[0][0] * (want - c * Xh[rows])
    for prec, tol in ((lib.F64, 1e-12), (lib.F32, 2e-5)):
        Z = X.clone()
        op.filter(Z, 1, a, b, aL, prec=prec, block=B)
        got = _gather_rows(Z, rows)
        assert np.max(np.abs(got - step)) <= tol * np.max(np.abs(step))


def test_c3_largest_complex_apply_sampled(ctx):
    s3 = workloads.config("c3", 7)
    s = s3.with_k(workloads.kpoints_mp4(s3.L)[0])
    op = lib.Operator(ctx, s)
    ref = fe.build_operator(s)
    X = _block(op.M, True, 103)
    Y = torch.zeros_like(X)
    op.apply(X, Y)
    rows = _rows(op.M, 40, 104)
    want = fe.apply_rows(ref, X.cpu().numpy(), rows)
    got = _gather_rows(Y, rows)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_c1_quadrature_potential_apply_sampled(ctx):
    s = workloads.config("c1")
    op = lib.Operator(ctx, s, potential="quadrature")
    ref = fe.build_operator(s)
    X = _block(op.M, False, 105)
    Y = torch.zeros_like(X)
    op.apply(X, Y)
    rows = _rows(op.M, 30, 106)
    Xh = X.cpu().numpy()
    Vq = dhm.gauss_potential(s)
    A0 = ref.cell_matrix()
    DX = ref.D[:, None] * Xh
    want = np.zeros((rows.size, B))
    for i, j in enumerate(rows):
        ce, lo = np.nonzero(ref.cells == j)
        Kl = dhm.cell_local_matrices(s, Vq[ce])
        acc = np.zeros(B)
        for n, (c, l) in enumerate(zip(ce, lo)):
            acc += (A0[l] + Kl[n, l]) @ DX[ref.cells[c]]
        want[i] = ref.D[j] * acc
    P = ref.hvec[:, None] * (ref.C.conj().T @ Xh)
    want += np.real(ref.C[rows] @ P)
    got = _gather_rows(Y, rows)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_c1_bf16_apply_sampled(ctx):
    # the BF16 scheme at full size: cell products on bf16-rounded scaled cell
    # matrices and bf16-rounded cell blocks, FP32 accumulation; potential and
    # projector terms on X as given (tolerance 2e-5 as in the small tests)
    s = workloads.config("c1")
    op = lib.Operator(ctx, s)
    ref = fe.build_operator(s)
    g = torch.Generator(device="cuda").manual_seed(107)
    X = torch.randn(op.M, B, dtype=torch.float32, device="cuda", generator=g)
    Y = torch.zeros_like(X)
    op.apply(X, Y, prec=lib.BF16)
    rows = _rows(op.M, 30, 108)
    Xh = X.cpu().numpy().astype(np.float64)
    A0 = ref.cell_matrix()
    want = np.zeros((rows.size, B))
    for i, j in enumerate(rows):
        ce, lo = np.nonzero(ref.cells == j)
        acc = np.zeros(B)
        for c, l in zip(ce, lo):
            nodes = ref.cells[c]
            Ac = fe.bf16_round(ref.D[nodes[l]] * A0[l] * ref.D[nodes])
            acc += Ac @ fe.bf16_round(Xh[nodes])
        want[i] = acc + ref.V[j] * Xh[j]
    P = ref.hvec[:, None] * (ref.C.conj().T @ Xh)
    want += np.real(ref.C[rows] @ P)
    got = _gather_rows(Y, rows).astype(np.float64)
    assert np.max(np.abs(got - want)) <= 2e-5 * np.max(np.abs(want))


def test_c3_largest_complex64_apply_sampled(ctx):
    s3 = workloads.config("c3", 7)
    s = s3.with_k(workloads.kpoints_mp4(s3.L)[0])
    op = lib.Operator(ctx, s)
    ref = fe.build_operator(s)
    g = torch.Generator(device="cuda").manual_seed(109)
    X = torch.randn(op.M, B, dtype=torch.complex64, device="cuda", generator=g)
    Y = torch.zeros_like(X)
    op.apply(X, Y, prec=lib.C64)
    rows = _rows(op.M, 30, 110)
    want = fe.apply_rows(ref, X.cpu().numpy().astype(np.complex128), rows)
    got = _gather_rows(Y, rows).astype(np.complex128)
    assert np.max(np.abs(got - want)) <= 2e-5 * np.max(np.abs(want))
