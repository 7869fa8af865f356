"""Pins of three oracle parts against values derived by hand or by an
independent construction:

* ``fe.bf16_round``: round-to-nearest-even to bfloat16 (8 significant bits),
  checked on values whose correct rounding is worked out by hand: ties to
  even in both directions, a carry into the exponent, negatives,
  subnormals and values already representable.
* ``fe.apply_cellwise_bf16``: the bf16 cell-product scheme (rounded scaled
  cell matrix D_c A0 D_c times the rounded cell block, potential on the
  unrounded block), checked on trilinear elements (p = 1), where the scaled
  cell matrix has a closed form: 1/(6h^2) on the diagonal, 0 between edge
  neighbours, -1/(24h^2) between face- and body-diagonal neighbours.
* The Bloch phase of the projector images, e^{-ik.(x_j - nL)} (Eq.
  nonlocalHamDiscrete with the Bloch form of Eq. contEigenBZ): a 2x2x2
  supercell at the Gamma point applied to a Bloch vector e^{ik.x} u(x) with
  k in {0, pi/L}^3 must give e^{ik.x} (H_nl(k) u)(x) exactly, node by node.
  The supercell operator has no phase at all, so the identity checks the
  phase (including the image term nL) against plain image sums.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import fe


# -- bf16 rounding --------------------------------------------------------

U = 2.0 ** -8   # half a bf16 ulp at 1


def _cases():
    # (input, expected) with the expected value worked out by hand; bf16
    # keeps 7 fraction bits, so the spacing at 1 is 2^-7 = 2U.
    tiny = 2.0 ** -133          # smallest positive bf16 subnormal (2^-126 * 2^-7)
    return [
        (1.0, 1.0),
        (1.0 + U, 1.0),                         # tie -> even fraction 0
        (1.0 + 3 * U, 1.0 + 4 * U),             # tie between fractions 1 and 2 -> 2
        (1.0 + U + 2.0 ** -20, 1.0 + 2 * U),    # just above the tie -> up
        (1.0 + U - 2.0 ** -20, 1.0),            # just below the tie -> down
        (2.0 - U, 2.0),                         # tie at fraction 127 -> carry into the exponent
        (2.0 - 3 * U, 2.0 - 4 * U),             # tie between 125 and 126 -> 126
        (-(1.0 + 3 * U), -(1.0 + 4 * U)),       # sign does not change the rounding of the magnitude
        (-(1.0 + U), -1.0),
        (2.0 ** 101 * (1.5 + U), 3.0 * 2.0 ** 100),      # 1.1000000|1 x 2^101: tie -> even (down)
        (0.1, 0.10009765625),                   # 1.6 x 2^-4: fraction .6 * 128 = 76.8 -> 77
        (1.0 / 3.0, 171.0 / 512.0),             # 1.0101010|10... -> up
        (2.0 ** -130, 2.0 ** -130),             # subnormal, representable
        (1.5 * tiny, 2 * tiny),                 # subnormal tie between 1 and 2 units -> 2
        (2.5 * tiny, 2 * tiny),                 # subnormal tie between 2 and 3 units -> 2
        (0.5 * tiny, 0.0),                      # tie between 0 and the smallest subnormal -> 0
        (0.75 * tiny, tiny),                    # above half a unit -> up
        (0.0, 0.0),
        (-0.0, 0.0),
    ]


@pytest.mark.parametrize("x,want", _cases())
def test_bf16_round_hand_derived(x, want):
    got = fe.bf16_round(np.array([x]))[0]
    assert got == want, (x, got, want)


def test_bf16_round_keeps_representable_values_and_is_idempotent():
    # every value with at most 8 significant bits is kept; rounding twice changes nothing
    rng = np.random.default_rng(5)
    mant = rng.integers(128, 256, size=1000).astype(np.float64)        # 8-bit significands
    ex = rng.integers(-40, 40, size=1000)
    x = np.ldexp(mant, ex) * np.where(rng.random(1000) < 0.5, -1.0, 1.0)
    assert np.array_equal(fe.bf16_round(x), x)
    y = rng.standard_normal(1000) * 10.0 ** rng.integers(-5, 5, size=1000)
    r = fe.bf16_round(y)
    assert np.array_equal(fe.bf16_round(r), r)
    # and the error is at most half a unit of the 8th significant bit
    assert np.all(np.abs(r - np.float32(y)) <= np.abs(np.float32(y)) * 2.0 ** -8 * (1 + 1e-12))


# -- the bf16 cell-product scheme on trilinear elements ----------------------

def test_apply_cellwise_bf16_trilinear_closed_form():
    # p = 1, 4^3 cells of side h = 1.5: every node lies in 8 cells, so
    # M_jj = 8 (h/2)^3 = h^3 and D_c A0 D_c = K^c / (2 h^3), whose entries are
    # 1/(6h^2) = 2/27 (diagonal), 0 (edge neighbours) and -1/(24h^2) = -1/54
    # (face and body diagonals).  Rounded to bf16 by hand: 2/27 = 1.185185 x 2^-4,
    # 0.185185 * 128 = 23.70 -> 24, so 1.1875 x 2^-4 = 0.07421875; 1/54 has the
    # same significand, 1.1875 x 2^-6 = 0.0185546875.  x = 1 + 3 2^-8 rounds to
    # 1 + 2^-6 (tie to even).
    h, nc = 1.5, 4
    s = workloads.System(L=h * nc, ncell=nc, p=1, pos=np.array([[2.2, 2.1, 1.9]]), Z=np.array([2.0]),
                         s=np.array([1.3]))
    op = fe.build_operator(s)
    n = nc
    j = 1 + n * (1 + n * 1)            # node (1, 1, 1)

    def node(ix, iy, iz):
        return ix % n + n * (iy % n + n * (iz % n))

    x = 1.0 + 3.0 * 2.0 ** -8
    X = np.zeros((op.M, 1))
    X[j, 0] = x
    Y = fe.apply_cellwise_bf16(op, X)[:, 0]
    rx = 1.0 + 2.0 ** -6
    diag, off = 0.07421875, -0.0185546875
    V = op.V
    assert abs(V[j]) > 0.1                          # the potential term is visible
    # diagonal: 8 cells, plus the potential on the unrounded value
    assert Y[j] == pytest.approx(8 * diag * rx + V[j] * x, abs=1e-15)
    # edge neighbours: zero coupling
    for d in [(1, 0, 0), (0, -1, 0), (0, 0, 1)]:
        assert abs(Y[node(1 + d[0], 1 + d[1], 1 + d[2])]) < 1e-15
    # face diagonals: 2 cells each; body diagonals: 1 cell
    assert Y[node(2, 2, 1)] == pytest.approx(2 * off * rx, abs=1e-15)
    assert Y[node(1, 0, 2)] == pytest.approx(2 * off * rx, abs=1e-15)
    assert Y[node(2, 0, 2)] == pytest.approx(off * rx, abs=1e-15)
    # nothing else is touched (only the node itself carries a potential term)
    touched = {node(1 + a, 1 + b, 1 + c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)}
    rest = np.array([i for i in range(op.M) if i not in touched])
    assert np.all(Y[rest] == 0.0)


def test_apply_cellwise_bf16_unit_cells_closed_form():
    # With h = 1 (D = 1) the scheme still rounds: the
    # trilinear D_c A0 D_c has entries 1/6 and -1/24, which bf16 does not hold;
    # their rounded values are 171/1024 and -171/4096 by hand (1/6 = 1.0101..b
    # x 2^-3).  Checking the whole column against those closed forms.
    s = workloads.System(L=3.0, ncell=3, p=1, pos=np.zeros((0, 3)), Z=np.zeros(0), s=np.zeros(0))
    op = fe.build_operator(s)
    X = np.zeros((op.M, 1))
    X[0, 0] = 1.0
    Y = fe.apply_cellwise_bf16(op, X)[:, 0]
    assert Y[0] == 8 * 171.0 / 1024.0
    assert Y[1 + 3 * (1 + 3 * 0)] == pytest.approx(2 * -171.0 / 4096.0, abs=1e-16)
    assert Y[1 + 3 * (1 + 3 * 1)] == pytest.approx(-171.0 / 4096.0, abs=1e-16)


# -- Bloch phase of the projector images --------------------------------------

def _prim_and_super():
    # primitive box L = 4 with 2 atoms whose projector support (6w > L) crosses
    # the boundary several times; the supercell repeats it 2x2x2
    Lp, ncp, p = 4.0, 2, 3
    pos = np.array([[0.3, 3.6, 2.0], [2.9, 1.1, 0.2]])
    Z = np.array([1.5, 2.5])
    sg = np.array([0.7, 0.9])
    w = np.array([1.2, 0.9])
    hs = np.array([1.3, -0.7])
    hp = np.array([-0.4, 1.1])
    prim = workloads.System(L=Lp, ncell=ncp, p=p, pos=pos, Z=Z, s=sg, has_proj=True, w=w, h_s=hs, h_p=hp)
    shifts = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=float) * Lp
    sup = workloads.System(L=2 * Lp, ncell=2 * ncp, p=p, pos=np.concatenate([pos + t for t in shifts]),
                           Z=np.tile(Z, 8), s=np.tile(sg, 8), has_proj=True, w=np.tile(w, 8),
                           h_s=np.tile(hs, 8), h_p=np.tile(hp, 8))
    return prim, sup


def _fold_map(n):
    # supercell node J -> (primitive node, supercell coordinate index)
    n2 = 2 * n
    I = np.arange(n2 ** 3)
    ix, iy, iz = I % n2, (I // n2) % n2, I // (n2 * n2)
    return (ix % n) + n * ((iy % n) + n * (iz % n)), ix, iy, iz


@pytest.mark.parametrize("kf", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (1, 1, 1)])
def test_bloch_phase_of_projectors_by_supercell_folding(kf):
    prim, sup = _prim_and_super()
    k = math.pi / prim.L * np.asarray(kf, dtype=float)
    opk = fe.build_operator(prim.with_k(k))
    ops = fe.build_operator(sup)
    assert not ops.is_complex
    n = prim.ncell * prim.p
    pm, ix, iy, iz = _fold_map(n)
    # the supercell's nodes are the primitive ones shifted by whole periods
    x1p = fe.node_coords_1d(prim.ncell, prim.p, prim.L)
    x1s = fe.node_coords_1d(sup.ncell, sup.p, sup.L)
    assert np.allclose(x1s, np.concatenate([x1p, x1p + prim.L]), atol=1e-14)
    xs = np.stack([x1s[ix], x1s[iy], x1s[iz]], axis=1)
    phase = np.exp(1j * (xs @ k))
    rng = np.random.default_rng(17)
    u = rng.standard_normal((opk.M, 3)) + 1j * rng.standard_normal((opk.M, 3))
    psi = phase[:, None] * u[pm]
    lhs = fe.apply_nonlocal(ops, psi)
    rhs = phase[:, None] * fe.apply_nonlocal(opk, u)[pm]
    scale = np.max(np.abs(rhs))
    assert scale > 1e-2                       # the projectors act
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * scale
    # the local potential and the lumped mass are periodic on the primitive box
    assert np.allclose(ops.V, opk.V[pm], atol=1e-13)
    assert np.allclose(ops.Mdiag, opk.Mdiag[pm], atol=1e-14)


def test_bloch_phase_without_image_term_would_differ():
    # The same identity fails for the phase e^{-ik.x_j} alone (image term nL
    # dropped): here built directly from the unphased image sums, to show that
    # the folding test above distinguishes the two readings on this system.
    prim, sup = _prim_and_super()
    k = math.pi / prim.L * np.array([1.0, 0.0, 0.0])
    op0 = fe.build_operator(prim)                      # k = 0: real image sums
    opk = fe.build_operator(prim.with_k(k))
    x1p = fe.node_coords_1d(prim.ncell, prim.p, prim.L)
    n = x1p.size
    I = np.arange(n ** 3)
    xp = np.stack([x1p[I % n], x1p[(I // n) % n], x1p[I // (n * n)]], axis=1)
    wrong = np.exp(-1j * (xp @ k))[:, None] * op0.C.toarray()
    right = opk.C.toarray()
    assert np.max(np.abs(wrong - right)) > 1e-2 * np.max(np.abs(right))
