"""Parity of the SCF pieces (chfsi_op_set_potential, chfsi_hartree,
chfsi_scf) with the oracle's SCF loop.

Tolerances.  Hartree: CG to a relative residual of 1e-12 on a problem with
condition number ~1e3, so 1e-9 relative on v_H; two solves of the same
density differ only in the order of the atomic dot-product sums (1e-11).  H~X after a potential
change: FP64 products, 1e-12.  SCF: the fixed point does not depend on the
eigensolver or the mixing path; both loops stop at an M-norm residual of
1e-9, the GPU one with ChFSI subspaces converged alongside, so densities
agree to 1e-6 of max rho, Ritz values and the Fermi level to 1e-6 Ha.
One k-point on a Bloch operator (no oracle loop at k != 0: parity unpinned
there): the Hartree solve equals Gamma's (it depends on the mesh only), and
the loops at k and -k, whose Hamiltonians are complex conjugates, agree to
the loop tolerance.
"""
import numpy as np
import pytest

import workloads
from oracle import fe
from oracle import scf as oscf

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2203_07820_amd as lib  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("nc,p,L", [(2, 4, 6.0), (3, 5, 7.5)])
def test_hartree_matches_oracle(ctx, nc, p, L):
    s = workloads.small_system(nc, p, 2, seed=3, L=L)
    op = lib.Operator(ctx, s)
    ref = fe.build_operator(s)
    rho = np.random.default_rng(4).uniform(0.01, 0.5, op.M)
    vh = torch.empty(op.M, dtype=torch.float64, device="cuda")
    it, rr = op.hartree(dev(rho), vh, tol=1e-12, maxit=5000)
    assert rr <= 1e-12
    want = oscf.hartree(ref, rho)
    got = vh.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-9 * np.max(np.abs(want))
    assert abs(float(np.sum(ref.Mdiag * got))) < 1e-9 * float(np.sum(ref.Mdiag * np.abs(got)))


def test_hartree_iteration_cap_and_repeat(ctx):
    # the device-side CG checks its residual every 8 iterations: a cap below
    # that stops at the cap unconverged; a converged solve reports a multiple
    # of 8; a repeated solve on the reused workspace gives the same potential
    s = workloads.small_system(3, 5, 2, seed=3, L=7.5)
    op = lib.Operator(ctx, s)
    ref = fe.build_operator(s)
    rho = np.random.default_rng(4).uniform(0.01, 0.5, op.M)
    vh = torch.empty(op.M, dtype=torch.float64, device="cuda")
    it, rr = op.hartree(dev(rho), vh, tol=1e-12, maxit=3)
    assert it == 3 and rr > 1e-12
    it, rr = op.hartree(dev(rho), vh, tol=1e-12, maxit=5000)
    assert it % 8 == 0 and rr <= 1e-12
    v1 = vh.cpu().numpy()
    it2, rr2 = op.hartree(dev(rho), vh, tol=1e-12, maxit=5000)
    assert it2 % 8 == 0 and rr2 <= 1e-12
    want = oscf.hartree(ref, rho)
    assert np.max(np.abs(vh.cpu().numpy() - v1)) <= 1e-11 * np.max(np.abs(want))
    assert np.max(np.abs(v1 - want)) <= 1e-9 * np.max(np.abs(want))


def test_set_potential_changes_the_operator(ctx):
    s = workloads.small_system(3, 4, 2, seed=5, has_proj=True)
    op = lib.Operator(ctx, s)
    ref = fe.build_operator(s)
    V = np.random.default_rng(6).uniform(-1.0, 1.0, op.M)
    op.set_potential(dev(V))
    H = oscf.hamiltonian(ref, V)
    X = np.random.default_rng(7).standard_normal((op.M, 9))
    Y = torch.zeros(op.M, 9, dtype=torch.float64, device="cuda")
    op.apply(dev(X), Y)
    want = H @ X
    assert np.max(np.abs(Y.cpu().numpy() - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("rr_mode", [0, 1, 2])
def test_scf_reaches_the_oracle_fixed_point(ctx, rr_mode):
    # rr_mode 0: full Rayleigh-Ritz and the density of the Ritz vectors;
    # 1, 2: spectrum-splitting Rayleigh-Ritz (FP64, mixed precision) and the
    # split density.  The fixed point does not depend on the route.
    s = workloads.small_system(2, 4, 2, seed=7, L=6.0)
    ref = oscf.scf(s, nstates=8, n_electrons=6.0, kT=0.01, beta=0.3, depth=4, tol=1e-9, maxit=80)
    assert ref.converged
    op = lib.Operator(ctx, s)
    M = op.M
    X = dev(workloads.start_block(M, 12, seed=8))
    m = fe.build_operator(s).Mdiag
    rho = dev(np.full(M, 6.0 / np.sum(m)))
    out = op.scf(X, rho, nwanted=8, n_buf=4, n_electrons=6.0, kT=0.01, m=20, beta=0.3, depth=4, tol=1e-9,
                 maxit=120, rr_mode=rr_mode)
    assert out["converged"], out["residuals"][-5:]
    got = rho.cpu().numpy()
    assert abs(float(np.sum(m * got)) - 6.0) < 1e-9
    assert np.max(np.abs(got - ref.rho)) <= 1e-6 * np.max(ref.rho)
    assert np.max(np.abs(out["theta"][:8] - ref.theta)) < 1e-6
    assert abs(out["mu"] - ref.mu) < 1e-6


def test_scf_rejects_bad_arguments(ctx):
    s = workloads.small_system(2, 3, 1, seed=9)
    op = lib.Operator(ctx, s)
    X = torch.randn(op.M, 6, dtype=torch.float64, device="cuda")
    rho = torch.full((op.M,), 0.01, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.ChfsiError):
        op.scf(X, rho, nwanted=4, n_buf=2, n_electrons=9.0, kT=0.01)     # more electrons than 2 nwanted
    opq = lib.Operator(ctx, s, potential="quadrature")
    with pytest.raises(lib.ChfsiError):
        opq.set_potential(rho)


def test_hartree_of_a_bloch_operator_equals_gamma(ctx):
    # the Hartree problem depends on the mesh only: a k != 0 operator of the
    # same system gives the Gamma operator's potential
    s0 = workloads.small_system(2, 4, 2, seed=3, L=6.0)
    sk = workloads.small_system(2, 4, 2, seed=3, L=6.0, k=(0.3, -0.1, 0.2))
    op0, opk = lib.Operator(ctx, s0), lib.Operator(ctx, sk)
    assert opk.is_complex and not op0.is_complex
    rho = np.random.default_rng(4).uniform(0.01, 0.5, op0.M)
    v0 = torch.empty(op0.M, dtype=torch.float64, device="cuda")
    vk = torch.empty(op0.M, dtype=torch.float64, device="cuda")
    op0.hartree(dev(rho), v0, tol=1e-12)
    opk.hartree(dev(rho), vk, tol=1e-12)
    assert np.max(np.abs(vk.cpu().numpy() - v0.cpu().numpy())) <= 1e-11 * np.max(np.abs(v0.cpu().numpy()))


@pytest.mark.parametrize("rr_mode", [0, 2])
def test_scf_at_k_and_minus_k_agree(ctx, rr_mode):
    # one k-point SCF on the complex Bloch operator: H(-k) is the complex
    # conjugate of H(k) (time reversal), so the loops at k and -k reach the
    # same density, Ritz values and Fermi level; the density holds N_e
    # electrons, and the upper Ritz values differ from the Gamma-point loop's
    def run(k):
        s = workloads.small_system(2, 4, 2, seed=7, L=6.0, k=k)
        op = lib.Operator(ctx, s)
        m = fe.build_operator(s).Mdiag
        X = dev(workloads.start_block(op.M, 12, seed=8, complex_=op.is_complex))
        rho = dev(np.full(op.M, 6.0 / np.sum(m)))
        out = op.scf(X, rho, nwanted=8, n_buf=4, n_electrons=6.0, kT=0.01, m=20, beta=0.3, depth=4, tol=1e-9,
                     maxit=120, rr_mode=rr_mode)
        return out, rho.cpu().numpy(), m
    k = (0.35, -0.2, 0.1)
    a, ra, m = run(k)
    b, rb, _ = run(tuple(-x for x in k))
    g, rg, _ = run((0.0, 0.0, 0.0))
    assert a["converged"] and b["converged"] and g["converged"]
    assert abs(float(np.sum(m * ra)) - 6.0) < 1e-9
    assert np.max(np.abs(ra - rb)) <= 1e-7 * np.max(ra)
    assert np.max(np.abs(a["theta"][:8] - b["theta"][:8])) < 1e-7
    assert abs(a["mu"] - b["mu"]) < 1e-7
    # the Bloch phase acts: the upper (delocalised) states move with k
    assert np.max(np.abs(a["theta"] - g["theta"])) > 1e-3


def test_scf_kpoints_pairs_and_single_point(ctx):
    # chfsi_scf_kpoints with k and -k at equal weights reaches the one-k
    # loop's fixed point (the two densities are equal by time reversal); a
    # single Gamma point through it is chfsi_scf; four k-points of a 2 x 2 x 1
    # shifted grid conserve the electron count and converge
    L, seed = 6.0, 7
    k = (0.35, -0.2, 0.1)

    def op_at(kk):
        return lib.Operator(ctx, workloads.small_system(2, 4, 2, seed=seed, L=L, k=kk))

    def block(op, sd):
        return dev(workloads.start_block(op.M, 12, seed=sd, complex_=op.is_complex))

    m = fe.build_operator(workloads.small_system(2, 4, 2, seed=seed, L=L)).Mdiag
    rho0 = np.full(m.size, 6.0 / np.sum(m))
    kw = dict(nwanted=8, n_buf=4, n_electrons=6.0, kT=0.01, m=20, tol=1e-9, maxit=120)
    # one k-point, the plain call
    opk = op_at(k)
    rho1 = dev(rho0)
    one = opk.scf(block(opk, 8), rho1, **kw)
    # k and -k
    ops = [op_at(k), op_at(tuple(-x for x in k))]
    rho2 = dev(rho0)
    two = ctx.scf_kpoints(ops, [block(ops[0], 8), block(ops[1], 9)], rho2, weights=[0.5, 0.5], **kw)
    assert one["converged"] and two["converged"]
    r1, r2 = rho1.cpu().numpy(), rho2.cpu().numpy()
    assert np.max(np.abs(r1 - r2)) <= 1e-7 * np.max(r1)
    assert abs(one["mu"] - two["mu"]) < 1e-7
    assert np.max(np.abs(two["theta"][0][:8] - two["theta"][1][:8])) < 1e-7
    # Gamma through the k-point call equals chfsi_scf
    # (bitwise, in the deterministic mode)
    op0 = op_at((0.0, 0.0, 0.0))
    rho3, rho4 = dev(rho0), dev(rho0)
    ctx.set_deterministic(True)
    a = op0.scf(block(op0, 8), rho3, **kw)
    b = ctx.scf_kpoints([op0], [block(op0, 8)], rho4, **kw)
    ctx.set_deterministic(False)
    assert a["iters"] == b["iters"] and a["mu"] == b["mu"]
    assert np.array_equal(rho3.cpu().numpy().view(np.uint64), rho4.cpu().numpy().view(np.uint64))
    # a shifted 2 x 2 x 1 grid
    g = 2.0 * np.pi / L
    ks = [(g * (i + 0.5) / 2 - g / 2, g * (j + 0.5) / 2 - g / 2, 0.0) for i in range(2) for j in range(2)]
    ops4 = [op_at(kk) for kk in ks]
    rho5 = dev(rho0)
    four = ctx.scf_kpoints(ops4, [block(o, 10 + i) for i, o in enumerate(ops4)], rho5, **kw)
    assert four["converged"]
    assert abs(float(np.sum(m * rho5.cpu().numpy())) - 6.0) < 1e-9
