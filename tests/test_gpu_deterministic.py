"""Deterministic assembly (chfsi_set_deterministic): the scatter of the cell
products into the global vector (Section 4.3, Eq. celldgemm) run colour
class by colour class, so that every node's sum is formed in a fixed order.

* Bitwise, deterministic path against itself: repeated H~.X, fused filter
  steps and apply_noalloc give the same bits (FP64, FP32, BF16 products,
  complex at k != 0; an odd side, 27 classes, and an even side, 8 classes).
* Bitwise, deterministic path against the atomic path, where the order
  cannot matter: a block supported on the interior nodes of one cell of a
  system without projectors.  Every other cell's product is exactly zero,
  so each node receives one nonzero contribution on both paths.
* Elsewhere the two paths add the same per-cell contributions (at most 8
  per node) in different orders: they differ by a few units of roundoff of
  the sum of the contributions' magnitudes, tested at 1e-13 relative to
  max|Y|, and both match the oracle to 1e-12 (the FP64 parity tolerance).
* The batched filter in this mode runs problem by problem and equals the
  individual deterministic filters bitwise; one cell per side (a cell that
  shares nodes with its own periodic images) is refused.
* The Hartree solve and the whole SCF loop give the same bits twice, and the
  atomic path agrees to the CG tolerance (1e-9 on v_H) and to the SCF
  tolerance (1e-6 on rho and mu).
"""
import numpy as np
import pytest

import workloads
from oracle import fe

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2203_07820_amd as lib  # noqa: E402

EINVAL = -1

CASES = [
    # (ncell, p, natoms, proj, k, seed): odd side (27 classes), even side (8)
    (3, 3, 2, True, (0.0, 0.0, 0.0), 11),
    (2, 5, 2, True, (0.0, 0.0, 0.0), 12),
    (4, 4, 3, True, (0.0, 0.0, 0.0), 13),
    (3, 4, 2, True, (0.1, -0.2, 0.3), 14),
]


@pytest.fixture()
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def _sys(nc, p, na, proj, k, seed):
    return workloads.small_system(nc, p, na, seed=seed, has_proj=proj, k=k)


def _apply(op, X, prec=None):
    Y = torch.zeros_like(X)
    op.apply(X, Y, prec=prec)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64 if a.dtype.itemsize % 8 == 0 else np.uint32)


def _relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("case", CASES)
def test_deterministic_apply_is_bitwise_repeatable_and_matches_atomic(ctx, case):
    s = _sys(*case)
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    X = workloads.start_block(op.M, 70, seed=5, complex_=op.is_complex)
    Xd = torch.from_numpy(X).cuda()
    Ya = _apply(op, Xd)
    ctx.set_deterministic(True)
    Yd1 = _apply(op, Xd)
    Yd2 = _apply(op, Xd)
    ctx.set_deterministic(False)
    assert np.array_equal(_bits(Yd1), _bits(Yd2))
    assert _relerr(Yd1, Ya) < 1e-13
    ref = H @ X
    assert _relerr(Yd1, ref) < 1e-12
    assert _relerr(Ya, ref) < 1e-12


@pytest.mark.parametrize("case", [CASES[0], CASES[3]])
def test_deterministic_filter_is_bitwise_repeatable(ctx, case):
    op = lib.Operator(ctx, _sys(*case))
    X0 = workloads.start_block(op.M, 40, seed=6, complex_=op.is_complex)
    b, _ = op.bounds(steps=20, seed=1)
    b = float(b)
    outs = []
    ctx.set_deterministic(True)
    for _ in range(2):
        Xd = torch.from_numpy(X0.copy()).cuda()
        op.filter(Xd, 6, 0.2 * b, b, -1.0)
        torch.cuda.synchronize()
        outs.append(Xd.cpu().numpy())
    ctx.set_deterministic(False)
    Xa = torch.from_numpy(X0.copy()).cuda()
    op.filter(Xa, 6, 0.2 * b, b, -1.0)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(outs[0]), _bits(outs[1]))
    assert _relerr(outs[0], Xa.cpu().numpy()) < 1e-11


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_deterministic_single_precision_is_bitwise_repeatable(ctx, prec):
    op = lib.Operator(ctx, _sys(*CASES[1]))
    X = torch.from_numpy(workloads.start_block(op.M, 64, seed=7)).float().cuda()
    p = lib.F32 if prec == "f32" else lib.BF16
    Ya = _apply(op, X, prec=p)
    ctx.set_deterministic(True)
    Y1 = _apply(op, X, prec=p)
    Y2 = _apply(op, X, prec=p)
    ctx.set_deterministic(False)
    assert np.array_equal(_bits(Y1), _bits(Y2))
    assert _relerr(Y1, Ya) < 1e-5


def test_one_nonzero_contribution_per_node_is_bitwise_equal_to_atomic(ctx):
    # no projectors; X nonzero only at the interior nodes of one cell
    nc, p = 3, 4
    s = workloads.small_system(nc, p, 2, seed=15, has_proj=False)
    op = lib.Operator(ctx, s)
    n = nc * p
    cx, cy, cz = 1, 2, 0
    rows = [((cx * p + a) % n) + n * (((cy * p + b) % n) + n * ((cz * p + c) % n))
            for c in range(1, p) for b in range(1, p) for a in range(1, p)]
    X = np.zeros((op.M, 50))
    X[rows, :] = workloads.start_block(len(rows), 50, seed=8)
    Xd = torch.from_numpy(X).cuda()
    Ya = _apply(op, Xd)
    ctx.set_deterministic(True)
    Yd = _apply(op, Xd)
    ctx.set_deterministic(False)
    assert np.count_nonzero(Ya) > 0
    assert np.array_equal(_bits(Ya), _bits(Yd))


def test_noalloc_in_deterministic_mode_equals_apply_bitwise(ctx):
    op = lib.Operator(ctx, _sys(*CASES[2]))
    X = torch.from_numpy(workloads.start_block(op.M, 33, seed=9)).cuda()
    ctx.set_deterministic(True)
    Y1 = _apply(op, X)
    Y2 = torch.zeros_like(X)
    ctx.check(ctx.lib.chfsi_apply_noalloc(op.h, lib._tptr(X), lib._tptr(Y2), 33, 33, lib.F64))
    torch.cuda.synchronize()
    ctx.set_deterministic(False)
    assert np.array_equal(_bits(Y1), _bits(Y2.cpu().numpy()))


def test_batched_filter_in_deterministic_mode_equals_individual_filters(ctx):
    ops = [lib.Operator(ctx, _sys(*CASES[0])), lib.Operator(ctx, _sys(3, 3, 3, True, (0.0, 0.0, 0.0), 16))]
    X0 = [workloads.start_block(op.M, 30, seed=20 + i) for i, op in enumerate(ops)]
    b = 80.0
    ctx.set_deterministic(True)
    Xs = [torch.from_numpy(x.copy()).cuda() for x in X0]
    ctx.filter_batched(ops, Xs, 5, [0.2 * b] * 2, [b] * 2, [-1.0] * 2, lib.F64, use_graph=True)
    ind = []
    for op, x in zip(ops, X0):
        Xd = torch.from_numpy(x.copy()).cuda()
        op.filter(Xd, 5, 0.2 * b, b, -1.0)
        ind.append(Xd)
    torch.cuda.synchronize()
    ctx.set_deterministic(False)
    for xb, xi in zip(Xs, ind):
        assert np.array_equal(_bits(xb.cpu().numpy()), _bits(xi.cpu().numpy()))


def test_one_cell_per_side_is_refused(ctx):
    op = lib.Operator(ctx, workloads.small_system(1, 3, 1, seed=17, has_proj=False, L=3.0))
    X = torch.from_numpy(workloads.start_block(op.M, 8, seed=10)).cuda()
    _apply(op, X)  # the atomic path takes it
    ctx.set_deterministic(True)
    Y = torch.zeros_like(X)
    rc = ctx.lib.chfsi_apply(op.h, lib._tptr(X), lib._tptr(Y), 8, 8, lib.F64)
    ctx.set_deterministic(False)
    assert rc == EINVAL
    assert "2 cells per side" in ctx.lib.chfsi_last_error(ctx.h).decode()


def test_deterministic_hartree_and_scf_are_bitwise_repeatable(ctx):
    # the Hartree solve (stiffness by colour class, CG sums in a fixed order)
    # and the whole SCF loop give the same bits twice; the atomic path agrees
    # to the CG tolerance
    s = workloads.small_system(2, 4, 2, seed=7, L=6.0)
    op = lib.Operator(ctx, s)
    M = op.M
    m = fe.build_operator(s).Mdiag
    rho0 = np.random.default_rng(4).uniform(0.01, 0.5, M)

    def hartree():
        vh = torch.zeros(M, dtype=torch.float64, device="cuda")
        it, rr = op.hartree(torch.from_numpy(rho0).cuda(), vh, tol=1e-12, maxit=5000)
        return it, vh.cpu().numpy()

    def scf():
        X = torch.from_numpy(workloads.start_block(M, 12, seed=8)).cuda()
        rho = torch.from_numpy(np.full(M, 6.0 / np.sum(m))).cuda()
        out = op.scf(X, rho, nwanted=8, n_buf=4, n_electrons=6.0, kT=0.01, m=20, tol=1e-9, maxit=120)
        return out, rho.cpu().numpy()

    it_a, vh_a = hartree()
    out_a, rho_a = scf()
    ctx.set_deterministic(True)
    it1, vh1 = hartree()
    it2, vh2 = hartree()
    out1, rho1 = scf()
    out2, rho2 = scf()
    ctx.set_deterministic(False)
    assert it1 == it2 and np.array_equal(_bits(vh1), _bits(vh2))
    assert np.max(np.abs(vh1 - vh_a)) <= 1e-9 * np.max(np.abs(vh_a))
    assert out1["converged"] and out2["converged"] and out_a["converged"]
    assert out1["iters"] == out2["iters"]
    assert np.array_equal(_bits(rho1), _bits(rho2))
    assert np.array_equal(_bits(out1["theta"]), _bits(out2["theta"]))
    assert np.array_equal(_bits(out1["residuals"]), _bits(out2["residuals"]))
    assert out1["mu"] == out2["mu"]
    assert np.max(np.abs(rho1 - rho_a)) <= 1e-6 * np.max(rho_a)
    assert abs(out1["mu"] - out_a["mu"]) < 1e-6
