"""Spectral finite-element operator of the Kohn-Sham problem, FP64 reference.

Test infrastructure only (see the package docstring).

What is computed, and where the paper defines it:

* Lagrange polynomials of order p on Gauss-Lobatto-Legendre (GLL) nodes
  (Section 2.3, the FE expansion of the wavefunctions).
* The discrete Hamiltonian of Section 2.3 (discrete H^loc: half the
  stiffness integral, the local potential and |k|^2/2 against the overlap,
  and the -i k.grad term; discrete H^nl: the separable projector sum).
  Stiffness and k.grad integrals use (p+1)-point Gauss-Legendre
  quadrature, which is exact for them on affine cells.
* The overlap matrix M evaluated with GLL quadrature, which makes it
  diagonal, and the Loewdin-transformed operator H~ = M^-1/2 H M^-1/2
  (Section 2.3, the standard Hermitian eigenproblem).
* The local potential and the projector vectors collocated at the nodes
  (GLL quadrature of their integrals against N_j).
* H~.X applied cell by cell (Section 4.3: extraction, cell products,
  assembly) for meshes too large to assemble.

Mesh: periodic cube [0, L)^3, ncell^3 cells of side h = L / ncell, order p,
n = ncell * p unique nodes per direction, M = n^3.  Node (ix, iy, iz) has
global id ix + n (iy + n iz) and x-coordinate (ix div p) h +
(1 + xi_(ix mod p)) h / 2.  Cell (cx, cy, cz) has id cx + ncell (cy + ncell
cz); its local node (a, b, c) has local id a + (p+1) (b + (p+1) c) and is the
global node ((cx p + a) mod n, ...).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import numpy.polynomial.legendre as npleg
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# 1D tables
# ---------------------------------------------------------------------------

def gll(p: int):
    """GLL nodes and weights on [-1, 1] for order p (p + 1 points).

    Nodes: the end points and the roots of P_p'; weights 2 / (p (p+1) P_p(x)^2).
    """
    if p < 1:
        raise ValueError("p >= 1")
    cp = np.zeros(p + 1)
    cp[p] = 1.0
    inner = npleg.legroots(npleg.legder(cp)) if p >= 2 else np.array([])
    x = np.concatenate(([-1.0], np.sort(np.real(inner)), [1.0]))
    Pp = npleg.legval(x, cp)
    w = 2.0 / (p * (p + 1) * Pp ** 2)
    return x, w


def gauss_legendre(nq: int):
    """nq-point Gauss-Legendre rule on [-1, 1] (exact to degree 2 nq - 1)."""
    return npleg.leggauss(nq)


def lagrange(nodes: np.ndarray, x: np.ndarray):
    """Values L[q, a] = l_a(x_q) and derivatives dL[q, a] = l_a'(x_q) of the
    Lagrange basis on ``nodes``, from the product definition."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = nodes.size
    L = np.ones((x.size, n))
    dL = np.zeros((x.size, n))
    for a in range(n):
        others = [b for b in range(n) if b != a]
        denom = np.prod([nodes[a] - nodes[b] for b in others])
        L[:, a] = np.prod([(x - nodes[b]) for b in others], axis=0) / denom
        acc = np.zeros(x.size)
        for c in others:
            term = np.ones(x.size)
            for b in others:
                if b != c:
                    term = term * (x - nodes[b])
            acc += term
        dL[:, a] = acc / denom
    return L, dL


@dataclasses.dataclass
class Tables1D:
    p: int
    h: float
    xi: np.ndarray       # GLL nodes
    wgll: np.ndarray     # GLL weights
    K1: np.ndarray       # int l_a' l_b' dx
    M1c: np.ndarray      # int l_a l_b dx (consistent mass, exact)
    G1: np.ndarray       # int l_a l_b' dx
    m1: np.ndarray       # GLL-lumped mass w_a h / 2


def tables_1d(p: int, h: float) -> Tables1D:
    xi, wg = gll(p)
    gq, gw = gauss_legendre(p + 1)
    Lq, dLq = lagrange(xi, gq)
    jac = h / 2.0
    # d/dx = (2/h) d/dxi ; dx = (h/2) dxi
    K1 = (dLq * gw[:, None]).T @ dLq * (1.0 / jac)
    M1c = (Lq * gw[:, None]).T @ Lq * jac
    G1 = (Lq * gw[:, None]).T @ dLq
    m1 = wg * jac
    return Tables1D(p, h, xi, wg, K1, M1c, G1, m1)


def kron3(z: np.ndarray, y: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Kronecker product with the x factor fastest (local id a + (p+1)(b + (p+1)c))."""
    return np.kron(z, np.kron(y, x))


@dataclasses.dataclass
class CellTables:
    K: np.ndarray        # stiffness (mcell x mcell)
    G: np.ndarray        # (3, mcell, mcell): int N_a d_alpha N_b
    m: np.ndarray        # lumped cell mass (mcell,)


def cell_tables(t: Tables1D) -> CellTables:
    K1, Mc, G1 = t.K1, t.M1c, t.G1
    K = kron3(Mc, Mc, K1) + kron3(Mc, K1, Mc) + kron3(K1, Mc, Mc)
    G = np.stack([kron3(Mc, Mc, G1), kron3(Mc, G1, Mc), kron3(G1, Mc, Mc)])
    m = kron3(t.m1, t.m1, t.m1)
    return CellTables(K, G, m)


# ---------------------------------------------------------------------------
# Mesh
# ---------------------------------------------------------------------------

def node_coords_1d(ncell: int, p: int, L: float) -> np.ndarray:
    h = L / ncell
    xi, _ = gll(p)
    n = ncell * p
    i = np.arange(n)
    return (i // p) * h + (1.0 + xi[i % p]) * h / 2.0


def node_coords(ncell: int, p: int, L: float) -> np.ndarray:
    """(M, 3) coordinates, global id ix + n (iy + n iz)."""
    x1 = node_coords_1d(ncell, p, L)
    n = x1.size
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.stack([x1[ix.ravel()], x1[iy.ravel()], x1[iz.ravel()]], axis=1)


def cell_nodes(ncell: int, p: int) -> np.ndarray:
    """(E, mcell) global node id of every local node of every cell."""
    n = ncell * p
    q = p + 1
    cz, cy, cx = np.meshgrid(np.arange(ncell), np.arange(ncell), np.arange(ncell), indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    c, b, a = np.meshgrid(np.arange(q), np.arange(q), np.arange(q), indexing="ij")
    a, b, c = a.ravel(), b.ravel(), c.ravel()
    gx = (cx[:, None] * p + a[None, :]) % n
    gy = (cy[:, None] * p + b[None, :]) % n
    gz = (cz[:, None] * p + c[None, :]) % n
    return (gx + n * (gy + n * gz)).astype(np.int64)


# ---------------------------------------------------------------------------
# Operator
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Operator:
    """Everything needed to apply H~(k) = D (K/2 - i k.G) D + diag(V + |k|^2/2)
    + sum_a sum_lm h_al c~_alm c~_alm^H, with D = M^-1/2 (GLL-lumped)."""
    ncell: int
    p: int
    L: float
    k: np.ndarray
    t1: Tables1D
    ct: CellTables
    cells: np.ndarray          # (E, mcell)
    Mdiag: np.ndarray          # (M,) lumped overlap
    D: np.ndarray              # (M,) M^-1/2
    V: np.ndarray              # (M,) nodal local potential
    C: Optional[sp.csr_matrix]  # (M, 4 na) projector vectors c~ (Loewdin scaled)
    hvec: Optional[np.ndarray]  # (4 na,) couplings h_s, h_p, h_p, h_p per atom
    _A0: Optional[np.ndarray] = None
    _asm: Optional[sp.csr_matrix] = None

    @property
    def M(self) -> int:
        return self.V.size

    @property
    def E(self) -> int:
        return self.cells.shape[0]

    @property
    def is_complex(self) -> bool:
        return bool(np.any(self.k != 0.0))

    @property
    def dtype(self):
        return np.complex128 if self.is_complex else np.float64

    def cell_matrix(self) -> np.ndarray:
        """Unscaled cell operator K^c/2 - i k.G^c (used with D on both sides)."""
        if self._A0 is None:
            A = 0.5 * self.ct.K.astype(self.dtype)
            if self.is_complex:
                A = A - 1j * np.einsum("a,aij->ij", self.k, self.ct.G)
            self._A0 = A
        return self._A0

    def assembly_matrix(self) -> sp.csr_matrix:
        """Sparse 0/1 matrix summing cell-local rows into global rows."""
        if self._asm is None:
            E, mc = self.cells.shape
            self._asm = sp.csr_matrix(
                (np.ones(E * mc), (self.cells.ravel(), np.arange(E * mc))),
                shape=(self.M, E * mc))
        return self._asm


def lumped_mass(ncell: int, p: int, L: float) -> np.ndarray:
    """Assembled GLL-lumped overlap diagonal M_jj = sum over cells of m^c."""
    t = tables_1d(p, L / ncell)
    ct = cell_tables(t)
    cells = cell_nodes(ncell, p)
    M = np.zeros(ncell ** 3 * p ** 3)
    np.add.at(M, cells.ravel(), np.tile(ct.m, cells.shape[0]))
    return M


def local_potential(sys, coords1d: np.ndarray) -> np.ndarray:
    """V_j = sum_a sum_images -Z_a exp(-|x_j - R_a - nL|^2 / (2 s_a^2)),
    image terms kept where the distance is at most 10 s_a."""
    n = coords1d.size
    L = sys.L
    V = np.zeros((n, n, n))  # [iz, iy, ix]
    for a in range(sys.natoms):
        R = sys.pos[a]
        s = float(sys.s[a])
        rc = 10.0 * s
        K = int(math.ceil(rc / L)) + 1
        for nz in range(-K, K + 1):
            for ny in range(-K, K + 1):
                for nx in range(-K, K + 1):
                    sh = np.array([nx, ny, nz], dtype=np.float64) * L
                    d1 = [coords1d - (R[i] + sh[i]) for i in range(3)]
                    idx = [np.nonzero(np.abs(d1[i]) <= rc)[0] for i in range(3)]
                    if any(ix.size == 0 for ix in idx):
                        continue
                    dz, dy, dx = np.meshgrid(d1[2][idx[2]], d1[1][idx[1]], d1[0][idx[0]], indexing="ij")
                    r2 = dx * dx + dy * dy + dz * dz
                    val = np.where(r2 <= rc * rc, -sys.Z[a] * np.exp(-r2 / (2.0 * s * s)), 0.0)
                    V[np.ix_(idx[2], idx[1], idx[0])] += val
    return V.ravel()


def projector_vectors(sys, coords1d: np.ndarray, Mdiag: np.ndarray, k: np.ndarray):
    """Loewdin-scaled collocated projector vectors (sparse M x 4 na) and the
    matching coupling vector.

    chi_s = n_s exp(-r^2/(2w^2)), chi_p,alpha = n_p r_alpha exp(-r^2/(2w^2)),
    unit L2 norm, zero beyond r = 6 w.  Column 4a + m holds
    c~_j = M_jj^(1/2) sum_n exp(-i k.(x_j - nL)) chi(x_j - R_a - nL).
    """
    n = coords1d.size
    L = sys.L
    cplx = bool(np.any(k != 0.0))
    rows, cols, vals = [], [], []
    hvec = np.zeros(4 * sys.natoms)
    for a in range(sys.natoms):
        w = float(sys.w[a])
        ns = (math.pi ** 1.5 * w ** 3) ** -0.5
        npn = (math.pi ** 1.5 * w ** 5 / 2.0) ** -0.5
        rc = 6.0 * w
        hvec[4 * a] = sys.h_s[a]
        hvec[4 * a + 1: 4 * a + 4] = sys.h_p[a]
        R = sys.pos[a]
        K = int(math.ceil(rc / L)) + 1
        for nz in range(-K, K + 1):
            for ny in range(-K, K + 1):
                for nx in range(-K, K + 1):
                    sh = np.array([nx, ny, nz], dtype=np.float64) * L
                    d1 = [coords1d - (R[i] + sh[i]) for i in range(3)]
                    idx = [np.nonzero(np.abs(d1[i]) <= rc)[0] for i in range(3)]
                    if any(ix.size == 0 for ix in idx):
                        continue
                    IZ, IY, IX = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
                    dx, dy, dz = d1[0][IX], d1[1][IY], d1[2][IZ]
                    r2 = dx * dx + dy * dy + dz * dz
                    keep = r2 <= rc * rc
                    if not np.any(keep):
                        continue
                    g = np.exp(-r2[keep] / (2.0 * w * w))
                    node = (IX + n * (IY + n * IZ))[keep]
                    xj = np.stack([coords1d[IX[keep]], coords1d[IY[keep]], coords1d[IZ[keep]]], axis=1)
                    if cplx:
                        phase = np.exp(-1j * ((xj - sh[None, :]) @ k))
                    else:
                        phase = 1.0
                    comps = [ns * g, npn * dx[keep] * g, npn * dy[keep] * g, npn * dz[keep] * g]
                    for m_, cv in enumerate(comps):
                        rows.append(node)
                        cols.append(np.full(node.size, 4 * a + m_))
                        vals.append(cv * phase)
    dtype = np.complex128 if cplx else np.float64
    if rows:
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        v = np.concatenate(vals).astype(dtype)
    else:
        r = c = np.zeros(0, dtype=np.int64)
        v = np.zeros(0, dtype=dtype)
    C = sp.csr_matrix((v, (r, c)), shape=(n ** 3, 4 * sys.natoms), dtype=dtype)
    C.sum_duplicates()
    C = sp.diags(np.sqrt(Mdiag)) @ C
    return sp.csr_matrix(C), hvec


def build_operator(sys, k=None) -> Operator:
    """Assemble everything that defines H~(k) for a ``workloads.System``."""
    if k is None:
        k = np.asarray(sys.k, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    h = sys.L / sys.ncell
    t = tables_1d(sys.p, h)
    ct = cell_tables(t)
    cells = cell_nodes(sys.ncell, sys.p)
    Mdiag = np.zeros(sys.ncell ** 3 * sys.p ** 3)
    np.add.at(Mdiag, cells.ravel(), np.tile(ct.m, cells.shape[0]))
    D = 1.0 / np.sqrt(Mdiag)
    x1 = node_coords_1d(sys.ncell, sys.p, sys.L)
    V = local_potential(sys, x1) if sys.natoms else np.zeros(Mdiag.size)
    C = hv = None
    if sys.has_proj and sys.natoms:
        C, hv = projector_vectors(sys, x1, Mdiag, k)
    return Operator(sys.ncell, sys.p, sys.L, k, t, ct, cells, Mdiag, D, V, C, hv)


def assemble(op: Operator) -> sp.csr_matrix:
    """Sparse H~(k), assembled globally: D (K/2 - i k.G) D + diag(V + |k|^2/2) + H_nl.
    Small meshes only (nnz grows like M (2p+1)^3)."""
    E, mc = op.cells.shape
    rows = np.repeat(op.cells, mc, axis=1).ravel()
    cols = np.tile(op.cells, (1, mc)).ravel()
    K = sp.csr_matrix((np.tile(op.ct.K.ravel(), E), (rows, cols)), shape=(op.M, op.M))
    H = 0.5 * K
    if op.is_complex:
        for al in range(3):
            if op.k[al] != 0.0:
                G = sp.csr_matrix((np.tile(op.ct.G[al].ravel(), E), (rows, cols)), shape=(op.M, op.M))
                H = H - 1j * op.k[al] * G
    Dm = sp.diags(op.D)
    H = Dm @ H @ Dm + sp.diags(op.V + 0.5 * float(op.k @ op.k))
    if op.C is not None:
        H = H + op.C @ sp.diags(op.hvec) @ op.C.conj().T
    return sp.csr_matrix(H)


def dense(op: Operator) -> np.ndarray:
    return assemble(op).toarray()


def apply_nonlocal(op: Operator, X: np.ndarray) -> np.ndarray:
    """sum_a sum_lm c~ h (c~^H X)  (Algorithm 4 collapsed to node level)."""
    if op.C is None:
        return np.zeros_like(X)
    P = op.C.conj().T @ X
    P = op.hvec[:, None] * P
    return op.C @ P


def apply_cellwise(op: Operator, X: np.ndarray, chunk: int = 512) -> np.ndarray:
    """Y = H~ X, computed as D . ASEMB{ A0 (D X)^c } + (V + |k|^2/2) X + H_nl X
    (Section 4.3: extraction, cell-level dense products, assembly)."""
    X = np.asarray(X)
    one = X.ndim == 1
    if one:
        X = X[:, None]
    dtype = np.result_type(X.dtype, op.dtype)
    A0 = op.cell_matrix()
    DX = op.D[:, None] * X
    Y = np.zeros((op.M, X.shape[1]), dtype=dtype)
    E = op.E
    for c0 in range(0, E, chunk):
        cs = op.cells[c0:c0 + chunk]
        Xc = DX[cs]                                  # (ncell, mcell, B)
        Yc = np.einsum("ij,cjb->cib", A0, Xc, optimize=True)
        idx = cs.ravel()
        Yflat = Yc.reshape(-1, X.shape[1])
        # scatter-add through a 0/1 assembly product (sums shared nodes)
        S = sp.csr_matrix((np.ones(idx.size), (idx, np.arange(idx.size))), shape=(op.M, idx.size))
        Y += S @ Yflat
    Y = op.D[:, None] * Y + (op.V + 0.5 * float(op.k @ op.k))[:, None] * X
    Y = Y + apply_nonlocal(op, X)
    return Y[:, 0] if one else Y


def apply_rows(op: Operator, X: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(H~ X)[rows, :] computed only from the cells that contain ``rows``
    (for spot checks on meshes too large to apply whole)."""
    rows = np.asarray(rows, dtype=np.int64)
    A0 = op.cell_matrix()
    dtype = np.result_type(X.dtype, op.dtype)
    out = np.zeros((rows.size, X.shape[1]), dtype=dtype)
    for r_i, j in enumerate(rows):
        ce, lo = np.nonzero(op.cells == j)
        acc = np.zeros(X.shape[1], dtype=dtype)
        for c, l in zip(ce, lo):
            nodes = op.cells[c]
            acc += A0[l] @ (op.D[nodes, None] * X[nodes])
        out[r_i] = op.D[j] * acc + (op.V[j] + 0.5 * float(op.k @ op.k)) * X[j]
    if op.C is not None:
        P = op.C.conj().T @ X
        P = op.hvec[:, None] * P
        out += op.C[rows] @ P
    return out


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (8-bit significand) with round-to-nearest-even, via
    float32; returned as float64.  Finite inputs only."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def apply_cellwise_bf16(op: Operator, X: np.ndarray, chunk: int = 512) -> np.ndarray:
    """H~ X of the bf16 filter scheme (real operators): the cell products use
    bf16-rounded scaled cell matrices D_c A0 D_c and bf16-rounded cell blocks
    X^c; the potential and projector terms use X as given.  Products and sums
    in FP64."""
    if op.is_complex:
        raise ValueError("bf16 scheme is defined for real operators")
    X = np.asarray(X, dtype=np.float64)
    A0 = op.cell_matrix()
    Y = np.zeros((op.M, X.shape[1]))
    for c0 in range(0, op.E, chunk):
        cs = op.cells[c0:c0 + chunk]
        for c in range(cs.shape[0]):
            nodes = cs[c]
            Ac = bf16_round(op.D[nodes, None] * A0 * op.D[None, nodes])
            Xc = bf16_round(X[nodes])
            np.add.at(Y, nodes, Ac @ Xc)
    Y = Y + op.V[:, None] * X + apply_nonlocal(op, X)
    return Y
