"""Pins of the oracle's finite-element operator against facts the
mathematics fixes (closed forms, textbook element matrices, invariants).

None of these re-types the oracle's own formulas: each compares it with an
independent value (a published quadrature rule, the exact integral of a
polynomial, the continuum spectrum of a free electron, a symmetry).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import fe


# -- 1D tables ---------------------------------------------------------------

def test_gll_p4_closed_form():
    # Lobatto rule with 5 points: nodes 0, +-sqrt(3/7), +-1; weights 32/45, 49/90, 1/10.
    x, w = fe.gll(4)
    r = math.sqrt(3.0 / 7.0)
    assert np.allclose(x, [-1, -r, 0, r, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_gll_weights_integrate_polynomials(p):
    # A (p+1)-point Lobatto rule integrates polynomials of degree 2p-1 exactly.
    x, w = fe.gll(p)
    for d in range(0, 2 * p):
        exact = 0.0 if d % 2 else 2.0 / (d + 1)
        assert abs(np.sum(w * x ** d) - exact) < 1e-14


def test_gauss_legendre_3pt_closed_form():
    g, w = fe.gauss_legendre(3)
    assert np.allclose(g, [-math.sqrt(0.6), 0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


def test_linear_element_textbook_matrices():
    # p = 1 on an element of length h: K = [[1,-1],[-1,1]]/h, M = h/6 [[2,1],[1,2]],
    # int N_a N_b' = [[-1/2, 1/2], [-1/2, 1/2]].
    h = 0.7
    t = fe.tables_1d(1, h)
    assert np.allclose(t.K1, np.array([[1, -1], [-1, 1]]) / h, atol=1e-14)
    assert np.allclose(t.M1c, h / 6 * np.array([[2, 1], [1, 2]]), atol=1e-15)
    assert np.allclose(t.G1, [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-15)
    assert np.allclose(t.m1, [h / 2, h / 2])


@pytest.mark.parametrize("p", [2, 4, 6])
def test_1d_matrices_integrate_interpolated_polynomials(p):
    # For polynomials u, v of degree <= p interpolated on the element [0, h]:
    # u^T M v = int u v, u^T K v = int u' v', u^T G v = int u v'.
    h = 1.3
    t = fe.tables_1d(p, h)
    xs = (1 + t.xi) * h / 2
    rng = np.random.default_rng(p)
    cu, cv = rng.standard_normal(p + 1), rng.standard_normal(p + 1)
    P = np.polynomial.Polynomial
    u, v = P(cu), P(cv)
    U, Vv = u(xs), v(xs)

    def integ(poly):
        ip = poly.integ()
        return ip(h) - ip(0.0)

    assert abs(U @ t.M1c @ Vv - integ(u * v)) < 1e-12 * max(1, abs(integ(u * v)))
    assert abs(U @ t.K1 @ Vv - integ(u.deriv() * v.deriv())) < 1e-11 * max(1, abs(integ(u.deriv() * v.deriv())))
    assert abs(U @ t.G1 @ Vv - integ(u * v.deriv())) < 1e-11 * max(1, abs(integ(u * v.deriv())))
    assert np.allclose(t.K1 @ np.ones(p + 1), 0, atol=1e-12)
    assert abs(t.M1c.sum() - h) < 1e-14
    # integration by parts on one element: G + G^T = e_p e_p^T - e_0 e_0^T
    B = np.zeros((p + 1, p + 1))
    B[-1, -1], B[0, 0] = 1, -1
    assert np.allclose(t.G1 + t.G1.T, B, atol=1e-13)


def test_mesh_numbering_is_a_partition_of_nodes():
    cells = fe.cell_nodes(3, 2)
    assert cells.shape == (27, 27)
    M = (3 * 2) ** 3
    counts = np.bincount(cells.ravel(), minlength=M)
    # vertex nodes of the periodic mesh are shared by 8 cells, interior ones by 1
    n = 6
    ix = np.arange(M) % n
    iy = (np.arange(M) // n) % n
    iz = np.arange(M) // (n * n)
    expect = (2 ** ((ix % 2 == 0).astype(int) + (iy % 2 == 0) + (iz % 2 == 0)))
    assert np.array_equal(counts, expect)


def test_lumped_mass_sums_to_volume():
    for (nc, p, L) in [(2, 3, 5.0), (3, 4, 7.0)]:
        M = fe.lumped_mass(nc, p, L)
        assert abs(M.sum() - L ** 3) < 1e-10 * L ** 3


# -- operator -----------------------------------------------------------------

def _free(nc, p, L, k=(0, 0, 0)):
    s = workloads.make_system(L, nc, p, 0, seed=0)
    return fe.build_operator(s, k=np.asarray(k, dtype=float))


def test_P1_zero_eigenvalue_with_sqrtM_vector():
    for p in (2, 3, 4):
        op = _free(2, p, 5.0)
        H = fe.dense(op)
        ev, Q = np.linalg.eigh(H)
        assert abs(ev[0]) < 1e-12
        v = np.sqrt(op.Mdiag)
        v /= np.linalg.norm(v)
        assert abs(abs(Q[:, 0] @ v) - 1.0) < 1e-10


def test_P2_constant_potential_shifts_spectrum():
    op = _free(2, 3, 5.0)
    ev0 = np.linalg.eigvalsh(fe.dense(op))
    op.V = np.full(op.M, -0.37)
    ev1 = np.linalg.eigvalsh(fe.dense(op))
    assert np.max(np.abs(ev1 - ev0 + 0.37)) < 1e-12


def _free_levels(L, k, nmax=4):
    G = 2 * math.pi / L
    r = range(-nmax, nmax + 1)
    lv = sorted(0.5 * ((G * a + k[0]) ** 2 + (G * b + k[1]) ** 2 + (G * c + k[2]) ** 2)
                for a in r for b in r for c in r)
    return np.array(lv)


def test_P3_free_electron_spectral_convergence():
    # V = 0, k = 0: eigenvalues -> (1/2)(2 pi / L)^2 |n|^2 with multiplicities
    # 1, 6, 12, 8 for |n|^2 = 0..3, and the error falls fast as p rises.
    L, nc = 5.0, 2
    exact = _free_levels(L, (0, 0, 0))[:27]
    errs = []
    for p in (2, 3, 4, 5, 6):
        ev = np.linalg.eigvalsh(fe.dense(_free(nc, p, L)))[:27]
        errs.append(np.max(np.abs(ev - exact)))
    for a, b in zip(errs, errs[1:]):
        assert b < a / 3
    assert errs[-1] < 1e-5
    first = np.linalg.eigvalsh(fe.dense(_free(nc, 6, L)))[1:7]
    assert np.max(np.abs(first - 0.5 * (2 * math.pi / L) ** 2)) < 1e-6
    # the cube of the first workload (L = 10, 4^3 cells, p = 4): first shell
    # 0.197392 Ha to better than 1e-7, and lambda_max of order 40 Ha
    ev = np.linalg.eigvalsh(fe.dense(_free(4, 4, 10.0)))
    assert np.max(np.abs(ev[1:7] - 0.5 * (2 * math.pi / 10.0) ** 2)) < 1e-7
    assert 30.0 < ev[-1] < 50.0


def test_P3k_free_electron_with_k_and_isospectral_minus_k():
    L, nc = 5.0, 2
    k = np.array([0.3, -0.2, 0.1])
    exact = _free_levels(L, k)[:20]
    errs = []
    for p in (3, 5):
        ev = np.linalg.eigvalsh(fe.dense(_free(nc, p, L, k)))[:20]
        errs.append(np.max(np.abs(ev - exact)))
    assert errs[1] < errs[0] / 10 and errs[1] < 1e-4
    e1 = np.linalg.eigvalsh(fe.dense(_free(nc, 4, L, k)))
    e2 = np.linalg.eigvalsh(fe.dense(_free(nc, 4, L, -k)))
    assert np.max(np.abs(e1 - e2)) < 1e-12


def test_operator_is_hermitian():
    s = workloads.small_system(2, 3, 2, seed=5, has_proj=True, k=(0.2, 0.1, -0.3))
    H = fe.dense(fe.build_operator(s))
    assert np.max(np.abs(H - H.conj().T)) < 1e-13 * np.max(np.abs(H))


def test_P7_translation_and_axis_swap_invariance():
    s = workloads.small_system(2, 3, 2, seed=11, has_proj=True)
    ev = np.linalg.eigvalsh(fe.dense(fe.build_operator(s)))
    h = s.L / s.ncell
    s2 = workloads.System(**{**s.__dict__, "pos": (s.pos + [h, 0, 0]) % s.L})
    ev2 = np.linalg.eigvalsh(fe.dense(fe.build_operator(s2)))
    s3 = workloads.System(**{**s.__dict__, "pos": s.pos[:, [1, 0, 2]].copy()})
    ev3 = np.linalg.eigvalsh(fe.dense(fe.build_operator(s3)))
    s4 = workloads.System(**{**s.__dict__, "pos": s.pos + [s.L, 0, -s.L]})
    ev4 = np.linalg.eigvalsh(fe.dense(fe.build_operator(s4)))
    for e in (ev2, ev3, ev4):
        assert np.max(np.abs(e - ev)) < 1e-11


def test_P8_cellwise_apply_matches_assembled_operator():
    s = workloads.small_system(3, 3, 3, seed=2, has_proj=True, k=(0.1, 0.25, -0.05))
    op = fe.build_operator(s)
    H = fe.assemble(op)
    X = workloads.start_block(op.M, 5, seed=9, complex_=True)
    Y1 = H @ X
    Y2 = fe.apply_cellwise(op, X, chunk=7)
    assert np.max(np.abs(Y1 - Y2)) < 1e-13 * np.max(np.abs(Y1))
    rows = np.array([0, 1, 17, op.M - 1])
    Y3 = fe.apply_rows(op, X, rows)
    assert np.max(np.abs(Y3 - Y1[rows])) < 1e-13 * np.max(np.abs(Y1))
    # the skew-symmetrised cell matrix assembles to the same operator
    Ge = np.einsum("a,aij->ij", op.k, op.ct.G)
    A_skew = 0.5 * op.ct.K - 0.5j * (Ge - Ge.T)
    E, mc = op.cells.shape
    rows_ = np.repeat(op.cells, mc, axis=1).ravel()
    cols_ = np.tile(op.cells, (1, mc)).ravel()
    Hs = sp.csr_matrix((np.tile(A_skew.ravel(), E), (rows_, cols_)), shape=(op.M, op.M))
    Dm = sp.diags(op.D)
    Hs = Dm @ Hs @ Dm + sp.diags(op.V + 0.5 * op.k @ op.k) + op.C @ sp.diags(op.hvec) @ op.C.conj().T
    assert abs(Hs - H).max() < 1e-13 * abs(H).max()


def test_gaussian_potential_quadrature_and_peak():
    # sum_j M_jj V_j is GLL quadrature of -Z exp(-r^2/2s^2): -Z (2 pi)^(3/2) s^3.
    s = workloads.make_system(12.0, 6, 6, 1, seed=3)
    s.pos[:] = [[5.5, 6.1, 4.9]]
    s.Z[:] = [2.5]
    s.s[:] = [0.9]
    op = fe.build_operator(s)
    integral = float(op.Mdiag @ op.V)
    assert abs(integral - (-2.5 * (2 * math.pi) ** 1.5 * 0.9 ** 3)) < 1e-6
    # an atom sitting on a node gives V = -Z there (images are beyond 10 s)
    x1 = fe.node_coords_1d(6, 6, 12.0)
    s.pos[:] = [[x1[7], x1[13], x1[20]]]
    op = fe.build_operator(s)
    j = 7 + 36 * (13 + 36 * 20)
    assert abs(op.V[j] + 2.5) < 1e-14
    assert op.V.min() >= -2.5 - 1e-14


def test_P12_projectors_normalised_orthogonal_and_low_rank():
    # c~ = M^(1/2) chi at the nodes, so |c~|^2 = sum_j M_jj chi(x_j)^2 is GLL
    # quadrature of int chi^2 = 1; s and p components are orthogonal by parity.
    s = workloads.make_system(16.0, 8, 6, 1, seed=4, has_proj=True)
    s.pos[:] = [[7.3, 8.2, 8.9]]
    s.w[:] = [1.3]
    op = fe.build_operator(s)
    C = op.C.toarray()
    G = C.T @ C
    assert np.max(np.abs(np.diag(G) - 1.0)) < 1e-4
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) < 1e-4
    # rank and trace of H_nl = sum h c c^H
    s2 = workloads.small_system(3, 3, 3, seed=8, has_proj=True)
    op2 = fe.build_operator(s2)
    Hnl = (op2.C @ sp.diags(op2.hvec) @ op2.C.T).toarray()
    assert np.linalg.matrix_rank(Hnl, tol=1e-10) <= 4 * s2.natoms
    tr = np.sum(op2.hvec * np.asarray(op2.C.multiply(op2.C).sum(axis=0)).ravel())
    assert abs(np.trace(Hnl) - tr) < 1e-12 * max(1.0, abs(tr))
    # a single s projector acting on X is h c (c^T X)
    X = workloads.start_block(op2.M, 3, seed=1)
    c0 = op2.C[:, 0].toarray()[:, 0]
    one = fe.Operator(**{**op2.__dict__, "C": op2.C[:, [0]], "hvec": op2.hvec[:1]})
    Y = fe.apply_nonlocal(one, X)
    assert np.allclose(Y, op2.hvec[0] * np.outer(c0, c0 @ X), atol=1e-14)
