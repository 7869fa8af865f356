"""Pins of the warm-start oracle: analytic gradients against central finite
differences (P13), the loss's invariances and limits, and the radial
features against a closed form for one atom."""
import math

import numpy as np

import workloads
from oracle import fe, mlp


def _setup(seed=0, M=60, din=32, hidden=16, dout=8):
    rng = np.random.default_rng(seed)
    params = mlp.init_params(din, hidden, dout, rng)
    for k in ("b1", "b2", "b3"):
        params[k] = 0.1 * rng.standard_normal(params[k].shape)
    Fn = rng.standard_normal((M, din))
    Q = np.linalg.qr(rng.standard_normal((M, dout)))[0]
    return params, Fn, Q


def _loss(params, Fn, Q):
    Y, _ = mlp.forward(params, Fn)
    return mlp.loss_and_grad_Y(Y, Q)[0]


def test_P13_gradients_match_central_differences():
    params, Fn, Q = _setup()
    Y, cache = mlp.forward(params, Fn)
    l, dY = mlp.loss_and_grad_Y(Y, Q)
    g = mlp.backward(params, cache, dY)
    vec = mlp.flatten(params)
    gvec = mlp.flatten(g)
    rng = np.random.default_rng(1)
    idx = rng.choice(vec.size, size=40, replace=False)
    h = 1e-6
    for i in idx:
        vp, vm = vec.copy(), vec.copy()
        vp[i] += h
        vm[i] -= h
        fd = (_loss(mlp.unflatten(vp, 32, 16, 8), Fn, Q) - _loss(mlp.unflatten(vm, 32, 16, 8), Fn, Q)) / (2 * h)
        assert abs(fd - gvec[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gvec[i])


def test_loss_gradient_wrt_Y_matches_differences():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((40, 6))
    Q = np.linalg.qr(rng.standard_normal((40, 6)))[0]
    l, dY = mlp.loss_and_grad_Y(Y, Q)
    h = 1e-6
    for _ in range(20):
        i, j = rng.integers(40), rng.integers(6)
        Yp, Ym = Y.copy(), Y.copy()
        Yp[i, j] += h
        Ym[i, j] -= h
        fd = (mlp.loss_and_grad_Y(Yp, Q)[0] - mlp.loss_and_grad_Y(Ym, Q)[0]) / (2 * h)
        assert abs(fd - dY[i, j]) <= 1e-7 * max(1.0, abs(fd))


def test_loss_invariances_and_limits():
    rng = np.random.default_rng(4)
    M, n = 80, 8
    Q = np.linalg.qr(rng.standard_normal((M, n)))[0]
    # a block spanning exactly span(Q) with orthogonal columns scaled equally:
    # first two terms 0, the coverage term only the ridge's d / (1 + d)
    R = np.linalg.qr(rng.standard_normal((n, n)))[0]
    assert abs(mlp.loss_and_grad_Y(3.0 * Q @ R, Q)[0] - 0.01 / 1.01) < 1e-14
    assert abs(mlp.loss_and_grad_Y(3.0 * Q @ R, Q, delta=0.0)[0]) < 1e-14
    # rotation / sign / scale invariance
    Y = rng.standard_normal((M, n))
    l0 = mlp.loss_and_grad_Y(Y, Q)[0]
    assert abs(mlp.loss_and_grad_Y(-2.5 * Y @ R, Q)[0] - l0) < 1e-12
    # a block orthogonal to span(Q): nothing of it inside, nothing of span(Q)
    # covered (first and third terms 1; orthonormal columns: second term 0)
    Yo = rng.standard_normal((M, n))
    Yo -= Q @ (Q.T @ Yo)
    Yo = np.linalg.qr(Yo)[0]
    assert abs(mlp.loss_and_grad_Y(Yo, Q)[0] - 2.0) < 1e-12
    # half of span(Q) plus half outside, orthonormal: half of the block
    # outside the target; the ridge eps = 0.01 (Y^T Y = I) leaves half of the
    # target covered to 1 / 1.01
    d = 0.01
    Yh = np.concatenate([Q[:, : n // 2] @ np.linalg.qr(rng.standard_normal((n // 2, n // 2)))[0],
                         Yo[:, : n // 2]], axis=1)
    assert abs(mlp.loss_and_grad_Y(Yh, Q)[0] - (0.5 + 1.0 - 0.5 / (1.0 + d))) < 1e-12
    # a block holding span(Q) and as much outside (2n orthonormal columns,
    # lam = 0): first term 1/2, third term d / (1 + d)
    Yc = np.concatenate([Q, Yo], axis=1)
    assert abs(mlp.loss_and_grad_Y(Yc, Q, lam=0.0)[0] - (0.5 + d / (1.0 + d))) < 1e-12
    # one target column scaled by 7: Y^T Y = diag(1, .., 49, .., 1), the
    # ridge is d ||Y||^2 / 2n, the first term 1 - ||Q^T Y||^2 / ||Y||^2
    Ys = Yc.copy()
    Ys[:, 3] *= 7.0
    s2 = float(np.sum(Ys ** 2))
    eps = d * s2 / (2 * n)
    first = 1.0 - float(np.sum((Q.T @ Ys) ** 2)) / s2
    third = 1.0 - ((n - 1) / (1.0 + eps) + 49.0 / (49.0 + eps)) / n
    assert abs(mlp.loss_and_grad_Y(Ys, Q, lam=0.0)[0] - (first + third)) < 1e-12


def test_features_single_atom_closed_form():
    s = workloads.make_system(30.0, 3, 2, 1, seed=0, has_proj=True)
    s.pos[:] = [[15.0, 15.0, 15.0]]
    s.Z[:] = [2.0]
    s.s[:] = [0.7]
    s.h_s[:] = [1.5]
    s.h_p[:] = [-0.5]
    pts = np.array([[15.0, 15.0, 15.0], [16.2, 15.0, 15.0], [15.0, 18.0, 19.0], [29.0, 29.0, 29.0]])
    F = mlp.features(s, pts)
    for i, x in enumerate(pts):
        r = np.linalg.norm(x - s.pos[0])
        g = np.exp(-((r - np.arange(8)) ** 2) / (2 * 0.25)) if r <= 10 else np.zeros(8)
        exp = np.concatenate([2.0 * g, 0.7 * g, 1.5 * g, -0.5 * g])
        assert np.allclose(F[i], exp, atol=1e-14)


def test_adam_first_step_moves_by_lr_sign():
    params, Fn, Q = _setup()
    Y, cache = mlp.forward(params, Fn)
    g = mlp.backward(params, cache, mlp.loss_and_grad_Y(Y, Q)[1])
    before = mlp.flatten(params).copy()
    mlp.adam_step(params, g, {}, lr=1e-3)
    step = mlp.flatten(params) - before
    gv = mlp.flatten(g)
    nz = np.abs(gv) > 1e-4
    assert np.allclose(step[nz], -1e-3 * np.sign(gv[nz]), rtol=1e-3, atol=1e-9)
