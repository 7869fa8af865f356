"""Solve history and the mixed-precision schedule, through the C ABI.

History: every recorded pass equals the oracle's pass-by-pass Ritz values
(1e-8 Ha, FP64) and the residual history its residual norms.  Mixed
schedule: a BF16 start is raised to FP32 and then FP64 and ends at the
FP64 accuracy (eigenvalues of the dense oracle operator to 1e-8 Ha), while
BF16 alone stalls at its rounding floor."""
import numpy as np
import pytest

import workloads
from oracle import chfsi as ochfsi
from oracle import fe

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2203_07820_amd as lib  # noqa: E402

LEVEL = {lib.BF16: 0, lib.F32: 1, lib.F64: 2}


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_history_follows_the_oracle_pass_by_pass(ctx):
    s = workloads.config("c0")
    op = lib.Operator(ctx, s)
    H = fe.assemble(fe.build_operator(s))
    N = 32
    X0 = workloads.start_block(op.M, N, seed=s.seed + 1_000_000)
    v0 = workloads.lanczos_start(op.M, seed=s.seed + 2_000_000)
    ref = ochfsi.solve(lambda v: H @ v, X0, N, m=20, block=32, v0=v0, passes=6)
    th, r, st = op.solve(dev(X0), N, m=20, block=32, fixed_passes=6, lanczos_v0=v0, history=True)
    h = st["history"]
    assert h["theta"].shape == (7, N)
    assert list(h["prec"]) == [-1] + [lib.F64] * 6
    assert np.all(np.diff(h["time_ms"]) > 0)
    for i in range(7):
        assert np.max(np.abs(h["theta"][i] - ref.history[i])) < 1e-8, i
        assert abs(h["max_resid"][i] - np.max(ref.resid_history[i])) < 1e-8 * max(1.0, h["max_resid"][i]), i
    assert np.array_equal(h["theta"][-1], th)
    assert h["max_resid"][-1] == st["max_resid"]
    assert st["final_prec"] == lib.F64 and st["prec_changes"] == 0


def _mixed_case():
    return workloads.small_system(3, 5, 3, seed=4, has_proj=True)


def test_mixed_schedule_reaches_fp64_accuracy(ctx):
    s = _mixed_case()
    op = lib.Operator(ctx, s)
    lam = np.linalg.eigvalsh(fe.dense(fe.build_operator(s)))
    N, nb = 16, 4
    X0 = workloads.start_block(op.M, N + nb, seed=21)
    v0 = workloads.lanczos_start(op.M, seed=22)
    th, r, st = op.solve(dev(X0), N, m=12, block=20, n_buf=nb, tol=1e-9, max_passes=80,
                         filter_prec=lib.BF16, prec_switch=True, lanczos_v0=v0, history=True)
    assert st["converged"]
    prec = st["history"]["prec"][1:]
    levels = [LEVEL[int(q)] for q in prec]
    assert levels[0] == 0 and levels == sorted(levels)       # BF16 first, never lowered
    assert st["final_prec"] == lib.F64 and st["prec_changes"] == 2
    assert np.max(np.abs(th[:N] - lam[:N])) < 1e-8


def test_bf16_alone_stalls_at_its_floor(ctx):
    s = _mixed_case()
    op = lib.Operator(ctx, s)
    N, nb = 16, 4
    X0 = workloads.start_block(op.M, N + nb, seed=21)
    v0 = workloads.lanczos_start(op.M, seed=22)
    _, _, st = op.solve(dev(X0), N, m=12, block=20, n_buf=nb, fixed_passes=25,
                        filter_prec=lib.BF16, lanczos_v0=v0, history=True)
    assert st["final_prec"] == lib.BF16 and st["prec_changes"] == 0
    assert st["max_resid"] > 1e-6      # the BF16 cell products limit the residual
    assert set(st["history"]["prec"][1:]) == {lib.BF16}


def test_batched_history_and_rejects_switch(ctx):
    systems = [workloads.small_system(2, 4, 2, seed=40 + i, has_proj=True) for i in range(2)]
    ops = [lib.Operator(ctx, s) for s in systems]
    N = 12
    Xs = [dev(workloads.start_block(op.M, N, seed=50 + i)) for i, op in enumerate(ops)]
    v0s = [workloads.lanczos_start(op.M, seed=60 + i) for i, op in enumerate(ops)]
    th, rs, stats = ctx.solve_batched(ops, Xs, N, m=10, block=N, filter_prec=lib.F64, fixed_passes=3,
                                      lanczos_v0=v0s, history=True)
    for q in range(2):
        h = stats[q]["history"]
        assert h["theta"].shape == (4, N)
        assert np.array_equal(h["theta"][-1], th[q])
        assert list(h["prec"]) == [-1, lib.F64, lib.F64, lib.F64]
        assert np.all(np.diff(h["time_ms"]) > 0)
    P = (lib._lib.Params * 1)()
    P[0].nwanted, P[0].m, P[0].block, P[0].fixed_passes, P[0].prec_switch = N, 10, N, 1, 1
    import ctypes as C
    theta_buf = np.zeros(N)
    out = (C.POINTER(C.c_double) * 1)(theta_buf.ctypes.data_as(C.POINTER(C.c_double)))
    rc = ctx.lib.chfsi_solve_batched(ctx.h, 1, (C.c_void_p * 1)(ops[0].h), P, (C.c_void_p * 1)(Xs[0].data_ptr()),
                                     (C.c_int64 * 1)(N), out, None, None, 0)
    assert rc == lib._lib.EINVAL
