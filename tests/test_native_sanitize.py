"""Sanitizer build of the host table code.

op_build.cpp (GLL/Gauss rules, cell matrices, D = M^-1/2, nodal potential,
projector tables: Section 2.3, Section 4.2, Algorithm 4) is host C++.  Here
it is compiled with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
together with a small driver (tests/native/tables_dump.cpp), run on systems
with p = 2..7, projectors whose support wraps around the periodic box and
k != 0, and its tables are compared with the oracle's.  Any sanitizer report
fails the run (halt_on_error, non-zero exit)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads
from oracle import fe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2203_07820_amd", "csrc", "op_build.cpp")
DRIVER = os.path.join(ROOT, "tests", "native", "tables_dump.cpp")

CASES = [
    # (ncell, p, natoms, k, seed, L)
    (2, 2, 1, (0, 0, 0), 1, None),
    (3, 3, 2, (0, 0, 0), 2, None),
    (2, 4, 3, (0.1, -0.2, 0.3), 3, None),
    (2, 5, 2, (0.25, 0.0, -0.1), 4, None),
    (2, 6, 2, (0, 0, 0), 5, 3.0),      # a small box: projector supports overlap their own images
    (2, 7, 1, (0.0, 0.3, 0.0), 6, None),
]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("san") / "tables_dump")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", SRC, DRIVER, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "hip_runtime" in r.stderr:
        pytest.skip("HIP headers not available for a host build")
    assert r.returncode == 0, r.stderr
    return out


def _write_system(s, path):
    na = s.natoms
    with open(path, "w") as f:
        k = [repr(float(v)) for v in s.k]
        f.write(f"{float(s.L)!r} {s.ncell} {s.p} {na} {1 if s.has_proj else 0} {k[0]} {k[1]} {k[2]}\n")
        for a in range(na):
            f.write(" ".join(repr(float(v)) for v in (*s.pos[a], s.Z[a], s.s[a], s.w[a], s.h_s[a], s.h_p[a])))
            f.write("\n")


@pytest.mark.parametrize("case", CASES)
def test_sanitized_tables_match_oracle(driver, tmp_path, case):
    nc, p, na, k, seed, L = case
    s = workloads.small_system(nc, p, na, seed=seed, has_proj=True, k=k, L=L)
    _write_system(s, tmp_path / "sys.txt")
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([driver, str(tmp_path / "sys.txt"), str(tmp_path)], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]

    def rd(name, dt):
        return np.fromfile(tmp_path / name, dtype=dt)

    M, E, mcell, cplx, npairs = (int(v) for v in open(tmp_path / "sizes").read().split())
    ref = fe.build_operator(s)
    assert (M, E, mcell) == (ref.M, ref.E, (p + 1) ** 3) and bool(cplx) == s.is_complex
    assert np.max(np.abs(rd("x1d", np.float64) - fe.node_coords_1d(nc, p, s.L))) < 1e-13
    assert np.max(np.abs(rd("dscale", np.float64) / ref.D - 1.0)) < 1e-14
    assert np.max(np.abs(rd("vdiag", np.float64) - (ref.V + 0.5 * ref.k @ ref.k))) < 1e-13
    Dc = ref.D[ref.cells[0]]
    Ge = np.einsum("a,aij->ij", ref.k, ref.ct.G)
    A = Dc[:, None] * (0.5 * ref.ct.K - 0.5j * (Ge - Ge.T)) * Dc[None, :]
    cre = rd("cell_re", np.float64).reshape(mcell, mcell)
    assert np.max(np.abs(cre - A.real)) < 1e-13 * np.max(np.abs(A.real))
    if cplx:
        cim = rd("cell_im", np.float64).reshape(mcell, mcell)
        assert np.max(np.abs(cim - A.imag)) < 1e-13 * max(np.max(np.abs(A.imag)), 1e-300)
    # node-level projector lists rebuild the oracle's Loewdin-scaled c~ (Eq. nonlocalHamDiscrete)
    ptr = rd("atom_ptr", np.int64)
    node = rd("atom_node", np.int32)
    val = rd("atom_val", np.float64)
    vw = 8 if cplx else 4
    val = val.reshape(-1, vw)
    val = val[:, 0::2] + 1j * val[:, 1::2] if cplx else val
    Cg = np.zeros((M, 4 * na), dtype=complex)
    for a in range(na):
        sl = slice(ptr[a], ptr[a + 1])
        assert np.all(np.diff(node[sl]) > 0)          # sorted, images merged
        Cg[node[sl], 4 * a:4 * a + 4] = val[sl]
    Cref = ref.C.toarray()
    assert np.max(np.abs(Cg - Cref)) < 1e-12 * np.max(np.abs(Cref))
    assert np.array_equal(rd("hcoef", np.float64), ref.hvec)
    # (cell, atom) pairs: sorted by cell, one per atom whose support touches the cell
    pp = rd("pair_ptr", np.int32)
    pa = rd("pair_atom", np.int32)
    assert pp[0] == 0 and pp[-1] == npairs == len(pa) and np.all(np.diff(pp) >= 0)
    for c in range(E):
        touching = {a for a in range(na) if np.any(Cref[ref.cells[c], 4 * a:4 * a + 4] != 0)}
        assert set(pa[pp[c]:pp[c + 1]].tolist()) == touching, c
