"""chfsi_apply_noalloc: H~.X with the projector scratch in the library's
fixed per-device array instead of context workspace.  Checked against
chfsi_apply on the same inputs (FP64, and complex at k != 0), on two calls in
a row, the second with a smaller input, so that whatever the first call left
in the shared scratch must not leak into the second; an input that needs
more than the fixed scratch is refused before any work."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2203_07820_amd as lib  # noqa: E402

EINVAL = -1


def _apply(op, X, noalloc):
    Y = torch.zeros_like(X)
    ncols, ld = X.shape[1], X.shape[1]
    prec = lib.C128 if op.is_complex else lib.F64
    f = op.ctx.lib.chfsi_apply_noalloc if noalloc else op.ctx.lib.chfsi_apply
    op.ctx.check(f(op.h, lib._tptr(X), lib._tptr(Y), ncols, ld, prec))
    torch.cuda.synchronize()
    return Y.cpu().numpy()


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.2, -0.1, 0.05)])
def test_noalloc_matches_apply_twice_second_smaller(k):
    ctx = lib.Context(0)
    big = lib.Operator(ctx, workloads.small_system(4, 5, 6, seed=61, has_proj=True, k=k))
    small = lib.Operator(ctx, workloads.small_system(2, 4, 2, seed=62, has_proj=True, k=k))
    cplx = big.is_complex
    for op, ncols, seed in ((big, 150, 1), (small, 37, 2)):
        X = torch.from_numpy(workloads.start_block(op.M, ncols, seed=seed, complex_=cplx)).cuda()
        ref = _apply(op, X, noalloc=False)
        got = _apply(op, X, noalloc=True)
        # same kernels, same inputs: only the order of the atomic assembly differs
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)), (op.M, ncols)
    big.close()
    small.close()
    ctx.close()


def test_noalloc_refuses_beyond_the_fixed_scratch():
    ctx = lib.Context(0)
    op = lib.Operator(ctx, workloads.small_system(6, 5, 24, seed=63, has_proj=True))
    ncols = 4096
    X = torch.zeros(op.M, ncols, dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    rc = ctx.lib.chfsi_apply_noalloc(op.h, lib._tptr(X), lib._tptr(Y), ncols, ncols, lib.F64)
    assert rc == EINVAL
    assert "fixed scratch" in ctx.lib.chfsi_last_error(ctx.h).decode()
    # chfsi_apply takes the same input through context workspace
    assert ctx.lib.chfsi_apply(op.h, lib._tptr(X), lib._tptr(Y), ncols, ncols, lib.F64) == 0
    torch.cuda.synchronize()
    op.close()
    ctx.close()
