"""Checkpoint and resume of a solve.  The state of ChFSI between passes is
the block of Ritz vectors and the filter bounds: the lower bounds a and a_L
come from the Ritz values (recomputed by the initial Rayleigh-Ritz of the
next call) and the upper bound b is passed in.  A solve stopped after k
passes, its block written to host memory (as a checkpoint file would hold
it) and restarted with the same b, must follow the uninterrupted solve:
the filter is linear in the block, so the restart's extra Rayleigh-Ritz
(a rotation of the Ritz basis within itself) leaves the next subspace
unchanged up to rounding.
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2203_07820_amd as lib  # noqa: E402


@pytest.fixture()
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.15, 0.05, -0.1)])
def test_solve_resumed_from_a_host_checkpoint_follows_the_uninterrupted_solve(ctx, k):
    s = workloads.small_system(3, 4, 3, seed=41, has_proj=True, k=k)
    op = lib.Operator(ctx, s)
    N, nbuf = 20, 6
    X0 = workloads.start_block(op.M, N + nbuf, seed=42, complex_=op.is_complex)
    b, _ = op.bounds(steps=20, seed=3)
    kw = dict(m=12, block=16, n_buf=nbuf, b_upper=b)

    full = torch.from_numpy(X0.copy()).cuda()
    th8, r8, st8 = op.solve(full, N, fixed_passes=8, **kw)

    part = torch.from_numpy(X0.copy()).cuda()
    th4, _, st4 = op.solve(part, N, fixed_passes=4, **kw)
    torch.cuda.synchronize()
    ckpt = part.cpu().numpy().copy()          # the checkpoint: block and b
    del part
    resumed = torch.from_numpy(ckpt).cuda()
    thr, rr, str_ = op.solve(resumed, N, fixed_passes=4, **kw)

    assert st4["b_upper"] == b and str_["b_upper"] == b and st8["b_upper"] == b
    assert st8["passes"] == 8 and st4["passes"] == 4 and str_["passes"] == 4
    # the checkpoint is a Ritz basis: its Ritz values are those it was saved with
    assert np.max(np.abs(th4 - th8)) > 1e-9          # not yet converged after 4 passes
    assert np.max(np.abs(thr[:N] - th8[:N])) < 1e-10
    assert np.max(np.abs(rr[:N] - r8[:N])) < 1e-8 * max(1.0, float(np.max(r8[:N])))
