"""Pins of the per-cell quadrature potential oracle (no GPU).

* A constant potential gives v0 times the consistent cell mass
  kron(M1, M1, M1) (the exact 1D mass matrices).
* A potential linear in x gives kron(M1, M1, X1) with the 1D first-moment
  matrix X1 integrated independently by a higher-order Gauss rule (the
  (p+1)-point rule is exact for degree 2p + 1).
* The Gauss-point potential equals the closed form evaluated point by point
  (atoms and periodic images looped in plain Python) at sampled points,
  which pins the point and cell ordering.
* No atoms: the operator equals the nodal one exactly; with atoms it is
  Hermitian, and its low eigenvalues approach those of the nodal-potential
  operator as p grows (both discretise the same continuum operator).
"""
import math

import numpy as np

import workloads
from oracle import dhm
from oracle import fe


def test_constant_potential_gives_consistent_mass():
    s = workloads.small_system(2, 4, 0, seed=1, L=5.0)
    h = s.L / s.ncell
    Vq = np.full((8, 125), 0.7)
    K = dhm.cell_local_matrices(s, Vq)
    t = fe.tables_1d(4, h)
    ref = 0.7 * fe.kron3(t.M1c, t.M1c, t.M1c)
    assert np.max(np.abs(K - ref[None])) < 1e-14 * np.max(np.abs(ref))


def test_linear_potential_gives_first_moment():
    p, nc, L = 3, 2, 4.0
    s = workloads.small_system(nc, p, 0, seed=2, L=L)
    h = L / nc
    g1 = dhm.gauss_points_1d(nc, p, L)
    q = p + 1
    # V = x at every Gauss point: x of point (cx, qx)
    Vq = np.empty((nc ** 3, q ** 3))
    for e in range(nc ** 3):
        cx = e % nc
        for pt in range(q ** 3):
            Vq[e, pt] = g1[cx * q + pt % q]
    K = dhm.cell_local_matrices(s, Vq)
    xi, _ = fe.gll(p)
    gq, gw = fe.gauss_legendre(p + 3)
    Lq, _ = fe.lagrange(xi, gq)
    t = fe.tables_1d(p, h)
    for e in (0, 1):   # cells with cx = 0 and cx = 1
        x0 = (e % nc) * h
        xq = x0 + (1.0 + gq) * h / 2.0
        X1 = (Lq * (gw * xq)[:, None]).T @ Lq * (h / 2.0)
        ref = fe.kron3(t.M1c, t.M1c, X1)
        assert np.max(np.abs(K[e] - ref)) < 1e-13 * np.max(np.abs(ref))


def test_gauss_potential_matches_closed_form_pointwise():
    s = workloads.small_system(3, 3, 3, seed=5, has_proj=False)
    Vq = dhm.gauss_potential(s)
    nc, q, L = s.ncell, s.p + 1, s.L
    h = L / nc
    gq, _ = fe.gauss_legendre(q)
    rng = np.random.default_rng(0)
    for _ in range(40):
        e = int(rng.integers(0, nc ** 3))
        pt = int(rng.integers(0, q ** 3))
        c = (e % nc, (e // nc) % nc, e // nc ** 2)
        iq = (pt % q, (pt // q) % q, pt // q ** 2)
        x = [c[i] * h + (1.0 + gq[iq[i]]) * h / 2.0 for i in range(3)]
        v = 0.0
        for a in range(s.natoms):
            sa = float(s.s[a])
            rc = 10.0 * sa
            K = int(math.ceil(rc / L)) + 1
            for nx in range(-K, K + 1):
                for ny in range(-K, K + 1):
                    for nz in range(-K, K + 1):
                        d = [x[0] - s.pos[a][0] - nx * L, x[1] - s.pos[a][1] - ny * L, x[2] - s.pos[a][2] - nz * L]
                        if max(abs(di) for di in d) > rc:
                            continue
                        r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
                        if r2 <= rc * rc:
                            v += -float(s.Z[a]) * math.exp(-r2 / (2.0 * sa * sa))
        assert abs(Vq[e, pt] - v) < 1e-13 * max(1.0, abs(v))


def test_operator_limits():
    s0 = workloads.small_system(2, 4, 0, seed=3, L=5.0)
    H0 = dhm.assemble_quadrature(s0).toarray()
    assert np.max(np.abs(H0 - fe.dense(fe.build_operator(s0)))) < 1e-13
    diffs = []
    for p in (3, 5):
        s = workloads.small_system(2, p, 2, seed=4, has_proj=True, L=6.0)
        Hq = dhm.assemble_quadrature(s).toarray()
        assert np.max(np.abs(Hq - Hq.T)) < 1e-13 * np.max(np.abs(Hq))
        lq = np.linalg.eigvalsh(Hq)[:6]
        ln = np.linalg.eigvalsh(fe.dense(fe.build_operator(s)))[:6]
        diffs.append(np.max(np.abs(lq - ln)))
    assert diffs[1] < diffs[0]
