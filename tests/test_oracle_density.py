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
