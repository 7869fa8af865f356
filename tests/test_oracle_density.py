"""Pins of the density / Fermi-level oracle (no GPU).

* Charge: sum_j rho_j M_jj = 2 sum_i w_i f_i = N_e for orthonormal Ritz
  vectors (the density integrates to the electron count under the lumped
  GLL quadrature).
* Free electron: the lowest state of -1/2 Laplacian on the periodic box is
  the constant function, whose Loewdin-basis vector is M^1/2 1 / sqrt(V);
  doubly occupied it gives rho = 2 / L^3 at every node.
* Rotation invariance: for fully occupied states the density depends only on
  the span (any orthonormal basis gives the same rho).
* Fermi level: the count condition, the zero-temperature limit (mu between
  the last occupied and the first empty level) and the symmetric two-level
  closed form (mu midway, f = 1/2 each, for one electron pair shared).
"""
import numpy as np

import workloads
from oracle import chfsi as ochfsi
from oracle import density as dens
from oracle import fe


def _eig(s, n):
    op = fe.build_operator(s)
    lam, V = np.linalg.eigh(fe.dense(op))
    return op, lam[:n], V[:, :n]


def test_charge_equals_electron_count():
    s = workloads.small_system(3, 3, 2, seed=5, has_proj=True)
    op, th, Psi = _eig(s, 12)
    for kT, ne in ((0.01, 16.0), (0.1, 15.3), (0.002, 9.0)):
        mu = dens.fermi_level(th, ne, kT)
        f = dens.occupations(th, mu, kT)
        rho = dens.density(Psi, 2.0 * f, op.Mdiag)
        assert abs(np.sum(rho * op.Mdiag) - ne) < 1e-10
        assert abs(dens.electron_count(th, mu, kT) - ne) < 1e-10


def test_free_electron_ground_state_density_is_uniform():
    for (nc, p, L) in ((3, 3, 6.0), (2, 5, 5.0)):
        s = workloads.small_system(nc, p, 0, seed=1, L=L)
        op, th, Psi = _eig(s, 1)
        assert abs(th[0]) < 1e-10
        rho = dens.density(Psi, np.array([2.0]), op.Mdiag)
        assert np.max(np.abs(rho - 2.0 / L ** 3)) < 1e-10 * (2.0 / L ** 3)


def test_density_of_full_shells_is_rotation_invariant():
    s = workloads.small_system(3, 3, 2, seed=6, has_proj=True)
    op, th, Psi = _eig(s, 10)
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((10, 10)))
    r1 = dens.density(Psi, np.full(10, 2.0), op.Mdiag)
    r2 = dens.density(Psi @ Q, np.full(10, 2.0), op.Mdiag)
    assert np.max(np.abs(r1 - r2)) < 1e-12 * np.max(r1)
    # and the spectrum-split form: an orthonormal basis of the span with
    # weight 2 plus the top (fractional) Ritz vectors with weight 2 (f - 1)
    f = np.ones(10)
    f[7:] = (0.8, 0.4, 0.1)
    direct = dens.density(Psi, 2.0 * f, op.Mdiag)
    Xo, _, _ = ochfsi.cholgs(Psi @ Q)
    split = dens.density(Xo, np.full(10, 2.0), op.Mdiag) + dens.density(Psi[:, 7:], 2.0 * (f[7:] - 1.0), op.Mdiag)
    assert np.max(np.abs(direct - split)) < 1e-12 * np.max(direct)


def test_fermi_level_limits_and_closed_form():
    th = np.array([-1.0, -0.5, 0.2, 0.3, 1.0])
    # zero-temperature limit: 4 electrons fill the two lowest levels
    mu = dens.fermi_level(th, 4.0, 1e-4)
    assert -0.5 < mu < 0.2
    # symmetric two-level system sharing one pair: mu at the midpoint, f = 1/2
    th2 = np.array([0.0, 0.4])
    mu2 = dens.fermi_level(th2, 2.0, 0.05)
    assert abs(mu2 - 0.2) < 1e-12
    assert np.allclose(dens.occupations(th2, mu2, 0.05), [0.5 + np.tanh(0.2 / 0.1) / 2, 0.5 - np.tanh(0.2 / 0.1) / 2])
    # weights (k-points) enter the count linearly
    w = np.array([0.25, 0.25, 0.25, 0.25, 0.25])
    mu3 = dens.fermi_level(th, 1.0, 0.01, weights=w)
    assert abs(dens.electron_count(th, mu3, 0.01, weights=w) - 1.0) < 1e-12


def test_gauss_density_free_electron_is_uniform():
    for (nc, p, L) in ((2, 4, 5.0), (3, 2, 4.0)):
        s = workloads.small_system(nc, p, 0, seed=2, L=L)
        op, th, Psi = _eig(s, 1)
        rho = dens.density_gauss(nc, p, L, Psi, np.array([2.0]))
        assert rho.shape == (nc ** 3, (p + 1) ** 3)
        assert np.max(np.abs(rho - 2.0 / L ** 3)) < 1e-10 * (2.0 / L ** 3)


def test_gauss_density_reproduces_cell_polynomials():
    # psi^ = g at the nodes with g a polynomial of degree <= p per axis: inside
    # every cell that does not wrap around the periodic box the interpolant is
    # g itself, so rho at the Gauss points equals w g(x_q)^2 (an anisotropic g
    # catches a transposed point order)
    nc, p, L = 3, 3, 6.0
    h = L / nc
    X = fe.node_coords(nc, p, L)
    g = lambda x, y, z: (1.0 + 0.3 * x - 0.05 * x ** 2 + 0.01 * x ** 3) * (2.0 - 0.1 * y ** 2) * (1.0 + 0.2 * z - 0.02 * z ** 3)
    Mdiag = fe.lumped_mass(nc, p, L)
    Psi = (np.sqrt(Mdiag) * g(X[:, 0], X[:, 1], X[:, 2]))[:, None]
    rho = dens.density_gauss(nc, p, L, Psi, np.array([0.7]))
    gq, _ = fe.gauss_legendre(p + 1)
    q1 = (1.0 + gq) * h / 2.0
    qz, qy, qx = np.meshgrid(q1, q1, q1, indexing="ij")
    checked = 0
    for cz in range(nc - 1):
        for cy in range(nc - 1):
            for cx in range(nc - 1):
                e = cx + nc * (cy + nc * cz)
                ref = 0.7 * g(cx * h + qx.ravel(), cy * h + qy.ravel(), cz * h + qz.ravel()) ** 2
                assert np.max(np.abs(rho[e] - ref)) < 1e-12 * np.max(np.abs(ref))
                checked += 1
    assert checked == 8


def test_gauss_density_integrates_to_consistent_mass_norms():
    # the (p+1)-point Gauss rule integrates |psi^|^2 exactly (degree 2p), so the
    # quadrature sum of rho equals sum_c w_c psi^_c^H M_cons psi^_c with the
    # consistent mass assembled cell by cell from the exact 1D mass matrices
    nc, p, L = 2, 4, 5.0
    s = workloads.small_system(nc, p, 2, seed=8, L=L, k=(0.3, -0.2, 0.1))
    op = fe.build_operator(s)
    rng = np.random.default_rng(4)
    Psi = rng.standard_normal((op.M, 5)) + 1j * rng.standard_normal((op.M, 5))
    w = np.array([2.0, 1.5, -0.3, 0.8, 2.0])
    rho = dens.density_gauss(nc, p, L, Psi, w)
    h = L / nc
    _, gw = fe.gauss_legendre(p + 1)
    Wq = fe.kron3(gw, gw, gw) * (h / 2.0) ** 3
    lhs = float(np.sum(rho * Wq[None, :]))
    t = fe.tables_1d(p, h)
    Mc = fe.kron3(t.M1c, t.M1c, t.M1c)
    Ph = op.D[:, None] * Psi
    rhs = 0.0
    for e in range(op.E):
        v = Ph[op.cells[e]]
        rhs += float(np.real(np.einsum("ac,ab,bc->c", v.conj(), Mc, v) @ w))
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
