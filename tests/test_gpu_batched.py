"""Batched path: many operators (uneven systems, k-points) in one persistent
launch per Chebyshev step, optionally captured in a hipGraph.  Each batched
result must equal the same problem solved alone (P14), and the batched
filter must match the oracle's filter.  FP64: 1e-12 relative for one filter
(only the order of the atomic assembly differs), 1e-10 Ha for Ritz values
after several passes."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

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


def _batch(k=(0.1, -0.2, 0.15)):
    # uneven periodic systems of the same order p = 3 (two of them share a
    # system at different k), complex Bloch operators
    specs = [(2, 2, 11), (3, 3, 12), (4, 2, 13)]
    out = []
    for (nc, na, seed) in specs:
        s = workloads.small_system(nc, 3, na, seed=seed, has_proj=True, k=k)
        out.append(s)
    out.append(out[0].with_k(np.array(k) * -0.5))
    return out


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("prec", ["c128", "f64"])
def test_batched_filter_matches_individual_and_oracle(ctx, use_graph, prec):
    k = (0.1, -0.2, 0.15) if prec == "c128" else (0.0, 0.0, 0.0)
    systems = _batch(k)
    ops = [lib.Operator(ctx, s) for s in systems]
    cplx = ops[0].is_complex
    ncols = [20, 37, 9, 33]
    Xs, refs, params = [], [], []
    for q, (s, op) in enumerate(zip(systems, ops)):
        H = fe.assemble(fe.build_operator(s))
        lam = np.linalg.eigvalsh(H.toarray())
        a, b, aL = lam[ncols[q]], lam[-1] * 1.05, lam[0]
        X = workloads.start_block(op.M, ncols[q], seed=50 + q, complex_=cplx)
        refs.append(ochfsi.cheb_filter(lambda v: H @ v, X, 8, a, b, aL))
        Xs.append(X)
        params.append((a, b, aL))
    P = lib.C128 if cplx else lib.F64
    Xd = [dev(X) for X in Xs]
    ctx.filter_batched(ops, Xd, 8, [p[0] for p in params], [p[1] for p in params], [p[2] for p in params], P,
                       block=16, use_graph=use_graph)
    for q in range(len(ops)):
        got = host(Xd[q])
        assert relerr(got, refs[q]) < 1e-11, q
        # the same block filtered alone
        Xi = dev(Xs[q])
        ops[q].filter(Xi, 8, *params[q], prec=P, block=16)
        assert relerr(got, host(Xi)) < 1e-12, q
    if use_graph:
        # replay the captured graph on fresh inputs with new intervals
        Xd2 = [dev(X) for X in Xs]
        ctx.filter_batched(ops, Xd2, 8, [p[0] * 1.01 for p in params], [p[1] for p in params],
                           [p[2] for p in params], P, block=16, use_graph=True)
        Xd3 = [dev(X) for X in Xs]
        ctx.filter_batched(ops, Xd3, 8, [p[0] * 1.01 for p in params], [p[1] for p in params],
                           [p[2] for p in params], P, block=16, use_graph=False)
        for q in range(len(ops)):
            assert relerr(host(Xd2[q]), host(Xd3[q])) < 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("col_tile", [64, 32])
def test_batched_real_filter_forced_col_tile(tmp_path, prec, col_tile):
    # real operators with the work item forced to 64 or 32 columns through the
    # tuning cache: blocks of 9 .. 37 columns (one ragged item of 64, or one or
    # two of 32), F64 and F32 (F32 with 64 columns takes the four-tile waves)
    systems = _batch((0.0, 0.0, 0.0))
    P = lib.F64 if prec == "f64" else lib.F32
    block = 40
    path = tmp_path / "tune.json"
    path.write_text('[\n{"key": "gfx950:p3:prec%d:B%d", "grid_per_cu": 0, "contiguous": 0, "col_tile": %d, '
                    '"ms": 1.0}\n]\n' % (P, block, col_tile))
    c = lib.Context(0)
    c.load_tuning(str(path))
    assert c.get_tuning(3, P, block)["col_tile"] == col_tile
    ops = [lib.Operator(c, s) for s in systems]
    ncols = [20, 37, 9, 33]
    Xs, refs, params = [], [], []
    for q, (s, op) in enumerate(zip(systems, ops)):
        H = fe.assemble(fe.build_operator(s))
        lam = np.linalg.eigvalsh(H.toarray())
        a, b, aL = lam[ncols[q]], lam[-1] * 1.05, lam[0]
        X = workloads.start_block(op.M, ncols[q], seed=70 + q)
        refs.append(ochfsi.cheb_filter(lambda v: H @ v, X, 8, a, b, aL))
        Xs.append(X)   # FP64 block; the F32 filter converts it and back
        params.append((a, b, aL))
    Xd = [dev(X) for X in Xs]
    c.filter_batched(ops, Xd, 8, [p[0] for p in params], [p[1] for p in params], [p[2] for p in params], P,
                     block=block, use_graph=False)
    tol = 1e-11 if prec == "f64" else 1e-4
    for q in range(len(ops)):
        assert relerr(host(Xd[q]), refs[q]) < tol, q
    for op in ops:
        op.close()
    c.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_solve_batched_equals_individual_solves(ctx, use_graph):
    systems = _batch()
    ops = [lib.Operator(ctx, s) for s in systems]
    nw = [12, 16, 10, 14]
    X0 = [workloads.start_block(op.M, nw[q] + 4, seed=70 + q, complex_=True) for q, op in enumerate(ops)]
    v0 = [workloads.lanczos_start(op.M, seed=80 + q, complex_=True) for q, op in enumerate(ops)]
    Xb = [dev(X) for X in X0]
    th, rs, st = ctx.solve_batched(ops, Xb, nw, m=10, block=8, filter_prec=lib.C128, n_buf=4, fixed_passes=4,
                                   lanczos_v0=v0, use_graph=use_graph)
    for q, op in enumerate(ops):
        Xi = dev(X0[q])
        thi, ri, sti = op.solve(Xi, nw[q], m=10, block=8, n_buf=4, fixed_passes=4, lanczos_v0=v0[q])
        assert st[q]["passes"] == 4
        assert np.max(np.abs(th[q] - thi)) < 1e-10
        assert np.max(np.abs(rs[q] - ri)) < 1e-9
        # and against the oracle iteration
        H = fe.assemble(fe.build_operator(systems[q]))
        ref = ochfsi.solve(lambda v: H @ v, X0[q], nw[q], m=10, block=8, v0=v0[q], passes=4)
        assert np.max(np.abs(th[q][:nw[q]] - ref.theta)) < 1e-8


@pytest.mark.parametrize("widest", [20, 70])
def test_solve_batched_real_equals_individual_solves(ctx, widest):
    # real operators; blocks of at most 64 columns take the subspace step of
    # all problems together (one Cholesky and one eigensolve launch), a
    # block of 70 columns makes every problem take its own
    systems = _batch((0.0, 0.0, 0.0))[:3]
    ops = [lib.Operator(ctx, s) for s in systems]
    nw = [12, widest - 4, 10]
    X0 = [workloads.start_block(op.M, nw[q] + 4, seed=170 + q) for q, op in enumerate(ops)]
    v0 = [workloads.lanczos_start(op.M, seed=180 + q) for q, op in enumerate(ops)]
    Xb = [dev(X) for X in X0]
    th, rs, st = ctx.solve_batched(ops, Xb, nw, m=10, block=16, filter_prec=lib.F64, n_buf=4, fixed_passes=3,
                                   lanczos_v0=v0, use_graph=False)
    for q, op in enumerate(ops):
        Xi = dev(X0[q])
        thi, ri, sti = op.solve(Xi, nw[q], m=10, block=16, n_buf=4, fixed_passes=3, lanczos_v0=v0[q])
        assert st[q]["passes"] == 3
        assert np.max(np.abs(th[q] - thi)) < 1e-10
        assert np.max(np.abs(rs[q] - ri)) < 1e-9
        # the lowest Ritz vectors up to sign (well separated Ritz values)
        Pb, Pi = host(Xb[q])[:, :6], host(Xi)[:, :6]
        sg = np.sign(np.sum(Pb * Pi, axis=0))
        assert relerr(Pb * sg[None, :], Pi) < 1e-8


def test_solve_batched_tolerance_retires_problems(ctx):
    systems = _batch()[:3]
    ops = [lib.Operator(ctx, s) for s in systems]
    nw = [8, 8, 8]
    X0 = [dev(workloads.start_block(op.M, 12, seed=90 + q, complex_=True)) for q, op in enumerate(ops)]
    th, rs, st = ctx.solve_batched(ops, X0, nw, m=12, block=12, filter_prec=lib.C128, n_buf=4, tol=1e-8,
                                   max_passes=40, use_graph=True)
    for q in range(3):
        assert np.max(rs[q][:8]) <= 1e-8
        H = fe.assemble(fe.build_operator(systems[q]))
        lam = np.linalg.eigvalsh(H.toarray())
        assert np.max(np.abs(th[q][:8] - lam[:8])) < 1e-9


def test_autotune_writes_cache_and_is_used(ctx, tmp_path):
    path = str(tmp_path / "tune.json")
    t = ctx.autotune(3, lib.C128, 16, cache_json=path)
    assert 0 <= t["grid_per_cu"] <= 4 and t["contiguous"] in (0, 1) and t["ms"] > 0
    assert t["col_tile"] in (32, 64)
    data = json.loads(open(path).read())
    assert any(e["key"] == "gfx950:p3:prec3:B16" for e in data)
    c2 = lib.Context(0)
    assert c2.get_tuning(3, lib.C128, 16)["ms"] == 0.0
    c2.load_tuning(path)
    t2 = c2.get_tuning(3, lib.C128, 16)
    assert (t2["grid_per_cu"], t2["contiguous"], t2["col_tile"]) == (t["grid_per_cu"], t["contiguous"], t["col_tile"])
    assert abs(t2["ms"] - t["ms"]) <= 1e-4 * t["ms"]
    c2.close()


def _c3_like():
    """Uneven p = 5 boxes with atoms and projectors, each at the 4 k-points of
    the reduced shifted Monkhorst-Pack grid: the shape of the batched k-point
    workload, at sizes the oracle filters in seconds."""
    out = []
    for (nc, na, seed) in [(2, 2, 21), (3, 3, 22)]:
        base = workloads.small_system(nc, 5, na, seed=seed, has_proj=True)
        for k in workloads.kpoints_mp4(base.L):
            out.append(base.with_k(k))
    return out


_C3_COLS = [24, 9, 40, 17, 33, 48, 12, 29]


@pytest.fixture(scope="module")
def c3_like_refs():
    """Oracle filters (degree 8, block 16) of every problem of the batch."""
    systems = _c3_like()
    refs, params, X0 = [], [], []
    for q, s in enumerate(systems):
        H = fe.assemble(fe.build_operator(s))
        lmax = float(spla.eigsh(H, k=1, which="LA", return_eigenvectors=False)[0])
        n = _C3_COLS[q]
        # any aL < a < b gives a well-defined filter to compare
        a, b, aL = 0.05 * lmax, lmax * 1.05, -0.1 * lmax
        X = workloads.start_block(s.M, n, seed=300 + q, complex_=True)
        refs.append(ochfsi.cheb_filter(lambda v: H @ v, X, 8, a, b, aL))
        params.append((a, b, aL))
        X0.append(X)
    return systems, refs, params, X0


# every launch shape of the batched cell kernel: one workgroup per item
# (grid_per_cu = 0), and persistent grids of 1, 2 and 4 workgroups per CU
# with contiguous or strided item assignment, each with the 64- and the
# 32-column work item (block 16 complex = 32 real columns: one 64-column item
# half padding, or one 32-column item; block 40 = 80 real columns: two items
# of 64 or three of 32, the last ragged)
TUNINGS = [(0, 1), (1, 1), (1, 0), (2, 1), (2, 0), (4, 1), (4, 0)]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("col_tile,block", [(64, 16), (32, 16), (64, 40), (32, 40)])
@pytest.mark.parametrize("tuning", TUNINGS)
def test_batched_p5_kpoints_every_launch_shape(c3_like_refs, tmp_path, tuning, col_tile, block, prec):
    systems, refs, params, X0 = c3_like_refs
    P = lib.C128 if prec == "c128" else lib.C64
    path = tmp_path / "tune.json"
    path.write_text('[\n{"key": "gfx950:p5:prec%d:B%d", "grid_per_cu": %d, "contiguous": %d, "col_tile": %d, '
                    '"ms": 1.0}\n]\n' % (P, block, tuning[0], tuning[1], col_tile))
    c = lib.Context(0)
    c.load_tuning(str(path))
    got_t = c.get_tuning(5, P, block)
    assert (got_t["grid_per_cu"], got_t["col_tile"]) == (tuning[0], col_tile)
    ops = [lib.Operator(c, s) for s in systems]
    Xd = [dev(X) for X in X0]
    c.filter_batched(ops, Xd, 8, [p[0] for p in params], [p[1] for p in params], [p[2] for p in params], P,
                     block=block, use_graph=True)
    tol_oracle, tol_alone = (1e-11, 1e-12) if prec == "c128" else (5e-5, 2e-5)
    for q in range(len(ops)):
        got = host(Xd[q])
        assert relerr(got, refs[q]) < tol_oracle, q
        Xi = dev(X0[q])
        ops[q].filter(Xi, 8, *params[q], prec=P, block=block)
        assert relerr(got, host(Xi)) < tol_alone, q
    for op in ops:
        op.close()
    c.close()
