"""Pins of the SCF oracle (no GPU).

* Hartree: for rho = rho_bar + A cos(2 pi x / L) the FE solution approaches
  the analytic 4 pi A (L / 2 pi)^2 cos(2 pi x / L), more closely at higher p.
* LDA exchange: v_x(8 rho) = 2 v_x(rho), v_x(0) = 0.
* Anderson mixing on a linear contraction x -> G x + c of dimension n with
  depth >= n reaches the fixed point in n + 2 steps (Anderson's method is a
  Krylov method on linear problems).
* SCF: convergence, charge conservation, and a fixed point that does not
  depend on the mixing parameters.
"""
import numpy as np

import workloads
from oracle import fe
from oracle import scf


def test_hartree_cosine_charge():
    errs = []
    for p in (4, 6):
        s = workloads.small_system(2, p, 0, seed=1, L=8.0)
        op = fe.build_operator(s)
        x = fe.node_coords(2, p, 8.0)[:, 0]
        A = 0.05
        rho = 0.3 + A * np.cos(2 * np.pi * x / 8.0)
        v = scf.hartree(op, rho)
        ref = 4 * np.pi * A * (8.0 / (2 * np.pi)) ** 2 * np.cos(2 * np.pi * x / 8.0)
        errs.append(np.max(np.abs(v - ref)) / np.max(np.abs(ref)))
        assert abs(np.sum(op.Mdiag * v)) < 1e-10
    assert errs[1] < errs[0] and errs[1] < 1e-4


def test_lda_exchange_scaling():
    r = np.array([0.0, 0.01, 0.3, 2.0])
    assert np.allclose(scf.lda_exchange(8.0 * r), 2.0 * scf.lda_exchange(r), rtol=1e-14, atol=0)
    assert scf.lda_exchange(np.array([0.0]))[0] == 0.0


def test_anderson_solves_linear_fixed_point():
    rng = np.random.default_rng(2)
    n = 6
    G = rng.standard_normal((n, n))
    G *= 0.6 / np.max(np.abs(np.linalg.eigvals(G)))
    c = rng.standard_normal(n)
    xs = np.linalg.solve(np.eye(n) - G, c)
    mix = scf.Anderson(0.5, n, np.ones(n))
    x = np.zeros(n)
    for _ in range(n + 2):
        x = mix.step(x, G @ x + c - x)
    assert np.max(np.abs(x - xs)) < 1e-9 * np.max(np.abs(xs))


def test_scf_converges_conserves_charge_and_is_mixing_independent():
    s = workloads.small_system(2, 4, 2, seed=7, L=6.0)
    r1 = scf.scf(s, nstates=8, n_electrons=6.0, kT=0.01, beta=0.3, depth=4)
    r2 = scf.scf(s, nstates=8, n_electrons=6.0, kT=0.01, beta=0.5, depth=2)
    assert r1.converged and r2.converged
    m = fe.build_operator(s).Mdiag
    assert abs(np.sum(m * r1.rho) - 6.0) < 1e-10
    assert np.max(np.abs(r1.rho - r2.rho)) < 1e-6 * np.max(r1.rho)
    assert abs(r1.mu - r2.mu) < 1e-7
