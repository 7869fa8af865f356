"""MI355X-native Chebyshev-filtered subspace iteration (ChFSI) on the
spectral finite-element Kohn-Sham Hamiltonian of DFT-FE 1.0
(arXiv 2203.07820).

This module is a thin binding of ``libchfsi.so`` (C ABI in
``include/chfsi.h``): it marshals torch tensors (device memory, streams)
and host arrays into the library's calls.  Every step of the method runs in
the library's HIP kernels; nothing here computes.
"""
from __future__ import annotations

import ctypes as C
import weakref
from typing import Optional

import numpy as np

from . import _lib
from ._lib import BF16, C64, C128, F32, F64, RHO_GAUSS, RHO_NODES  # noqa: F401

__all__ = ["ChfsiError", "Context", "Operator", "Network", "features", "initial_block", "fermi_level", "F64",
           "F32", "BF16", "C128", "C64", "RHO_NODES", "RHO_GAUSS", "load"]


class ChfsiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chfsi error {code}: {msg}")
        self.code = code


def load():
    return _lib.load()


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _tptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(0)
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _bptr(t) -> C.c_void_p:
    """Device pointer of a row-major block that may be a column slice of a
    wider one (unit column stride, row stride = ld)."""
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if t.dim() == 2 and t.stride(1) != 1 or t.dim() == 1 and not t.is_contiguous():
        raise ValueError("block rows must be contiguous (unit column stride)")
    return C.c_void_p(t.data_ptr())


def _ld_cols(t):
    """(ncols, ld) in logical entries of a row-major block tensor."""
    if t.dim() == 1:
        return 1, 1
    if t.dim() != 2:
        raise ValueError("block tensors are 2-D (M x ld)")
    return t.shape[1], t.stride(0)


def _attach_history(p, ncols: int, fixed_passes: int, max_passes: int):
    """Host arrays for the per-pass history of one solve, attached to Params p."""
    n = (fixed_passes if fixed_passes > 0 else (max_passes if max_passes > 0 else 100)) + 1
    h = {"time_ms": np.zeros(n), "max_resid": np.zeros(n), "prec": np.zeros(n, dtype=np.int32),
         "theta": np.zeros((n, ncols))}
    p.hist_len = n
    p.hist_time_ms = _dptr(h["time_ms"])
    p.hist_max_resid = _dptr(h["max_resid"])
    p.hist_prec = h["prec"].ctypes.data_as(C.POINTER(C.c_int32))
    p.hist_theta = _dptr(h["theta"])
    return h


def _trim_history(h, passes: int):
    return {k: v[:passes + 1].copy() for k, v in h.items()}


class Context:
    """A library context bound to one device and one HIP stream (torch's
    current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = _lib.load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        rc = self.lib.chfsi_ctx_create(C.byref(h), int(device), C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise ChfsiError(rc, self.lib.chfsi_last_error(None).decode())
        self.h = h
        self.device = device
        # operators must be destroyed before their context
        self._ops = weakref.WeakSet()

    def check(self, rc: int, allow=(0,)):
        if rc not in allow:
            raise ChfsiError(rc, self.lib.chfsi_last_error(self.h).decode())
        return rc

    def sync(self):
        self.check(self.lib.chfsi_sync(self.h))

    def set_timing(self, enable: bool):
        self.check(self.lib.chfsi_set_timing(self.h, 1 if enable else 0))

    def set_deterministic(self, enable: bool):
        """H~.X assembled colour class by colour class (bitwise reproducible)."""
        self.check(self.lib.chfsi_set_deterministic(self.h, 1 if enable else 0))

    def kernel_time(self, reset: bool = True):
        """(total ms, launches, algorithmic flops) of the timed cell-kernel launches."""
        ms, n, fl = C.c_double(), C.c_int64(), C.c_double()
        self.check(self.lib.chfsi_kernel_time(self.h, C.byref(ms), C.byref(n), C.byref(fl), 1 if reset else 0))
        return ms.value, n.value, fl.value

    # -- batched ----------------------------------------------------------
    def filter_batched(self, ops, Xs, m: int, a, b, aL, prec: int, block: int = 0, use_graph: bool = False):
        n = len(ops)
        VP = C.c_void_p * n
        I64 = C.c_int64 * n
        D = C.c_double * n
        cols = [_ld_cols(X) for X in Xs]
        self.check(self.lib.chfsi_filter_batched(
            self.h, n, VP(*[o.h for o in ops]), VP(*[_tptr(X) for X in Xs]), I64(*[c[0] for c in cols]),
            I64(*[c[1] for c in cols]), int(m), D(*a), D(*b), D(*aL), int(prec), int(block), 1 if use_graph else 0))

    def solve_batched(self, ops, Xs, nwanted, m: int, block: int, filter_prec: int, n_buf=0, fixed_passes: int = 0,
                      tol: float = 0.0, max_passes: int = 100, lanczos_v0=None, b_upper=None, use_graph: bool = True,
                      history: bool = False):
        """chfsi_solve_batched; nwanted / n_buf / lanczos_v0 / b_upper may be per-problem lists.
        With history=True each stats entry carries a per-pass "history" (see Operator.solve)."""
        n = len(ops)

        def per(x):
            return list(x) if isinstance(x, (list, tuple)) else [x] * n

        nw, nb, v0s, bs = per(nwanted), per(n_buf), per(lanczos_v0), per(b_upper)
        P = (_lib.Params * n)()
        keep = []
        for q in range(n):
            p = P[q]
            p.nwanted, p.n_buf, p.m, p.block = nw[q], nb[q], m, block
            p.fixed_passes, p.max_passes, p.tol = fixed_passes, max_passes, tol
            p.filter_prec, p.lanczos_steps = int(filter_prec), 20
            p.b_upper = float(bs[q]) if bs[q] is not None else 0.0
            if v0s[q] is not None:
                v = np.ascontiguousarray(v0s[q])
                v = np.ascontiguousarray(v.view(np.float64) if np.iscomplexobj(v) else v, dtype=np.float64)
                keep.append(v)
                p.lanczos_v0 = _dptr(v)
        cols = [_ld_cols(X) for X in Xs]
        for q in range(n):
            if cols[q][0] != nw[q] + nb[q]:
                raise ValueError("X must have nwanted + n_buf columns")
        hists = [_attach_history(P[q], cols[q][0], fixed_passes, max_passes) if history else None
                 for q in range(n)]
        th = [np.zeros(cols[q][0]) for q in range(n)]
        rs = [np.zeros(cols[q][0]) for q in range(n)]
        PD = C.POINTER(C.c_double) * n
        st = (_lib.Stats * n)()
        VP = C.c_void_p * n
        rc = self.lib.chfsi_solve_batched(self.h, n, VP(*[o.h for o in ops]), P, VP(*[_tptr(X) for X in Xs]),
                                          (C.c_int64 * n)(*[c[1] for c in cols]), PD(*[_dptr(t) for t in th]),
                                          PD(*[_dptr(r) for r in rs]), st, 1 if use_graph else 0)
        self.check(rc, allow=(0, 1))
        stats = [{f: getattr(st[q], f) for f, _ in _lib.Stats._fields_} for q in range(n)]
        for q in range(n):
            if hists[q] is not None:
                stats[q]["history"] = _trim_history(hists[q], stats[q]["passes"])
        return th, rs, stats

    def scf_kpoints(self, ops, Xs, rho, nwanted: int, n_buf: int, n_electrons: float, kT: float, weights=None,
                    m: int = 20, block: int = 0, beta: float = 0.3, depth: int = 4, tol: float = 1e-8,
                    maxit: int = 60, rr_mode: int = 2):
        """chfsi_scf_kpoints: one SCF loop over the k-points `ops` (one mesh),
        blocks `Xs` (device tensors), weights (None: equal)."""
        n = len(ops)
        VP = C.c_void_p * n
        I64 = C.c_int64 * n
        lds = []
        for X in Xs:
            ncols, ld = _ld_cols(X)
            if ncols != nwanted + n_buf:
                raise ValueError("each X must have nwanted + n_buf columns")
            lds.append(ld)
        ths = [np.zeros(nwanted + n_buf) for _ in range(n)]
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        hist = np.zeros(maxit)
        mu, it = C.c_double(), C.c_int32()
        rc = self.check(self.lib.chfsi_scf_kpoints(
            self.h, n, VP(*[o.h for o in ops]), VP(*[_tptr(X) for X in Xs]), I64(*lds),
            None if w is None else C.c_void_p(w.ctypes.data), int(nwanted), int(n_buf), int(m), int(block), int(rr_mode),
            float(n_electrons), float(kT), float(beta), int(depth), float(tol), int(maxit), _tptr(rho),
            VP(*[C.c_void_p(t.ctypes.data) for t in ths]), C.byref(mu), _dptr(hist), C.byref(it)), allow=(0, 1))
        return {"theta": ths, "mu": mu.value, "iters": it.value, "residuals": hist[:it.value],
                "converged": rc == 0}

    def autotune(self, p: int, prec: int, block: int, cache_json: Optional[str] = None):
        self.check(self.lib.chfsi_autotune(self.h, cache_json.encode() if cache_json else None, int(p), int(prec),
                                           int(block)))
        return self.get_tuning(p, prec, block)

    def load_tuning(self, cache_json: str):
        self.check(self.lib.chfsi_load_tuning(self.h, cache_json.encode()))

    def get_tuning(self, p: int, prec: int, block: int):
        g, c, ct, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        self.check(self.lib.chfsi_get_tuning(self.h, int(p), int(prec), int(block), C.byref(g), C.byref(c),
                                             C.byref(ct), C.byref(ms)))
        return {"grid_per_cu": g.value, "contiguous": c.value, "col_tile": ct.value, "ms": ms.value}

    def close(self):
        if getattr(self, "h", None):
            for op in list(getattr(self, "_ops", ())):
                op.close()
            self.check(self.lib.chfsi_ctx_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """The operator H~(k) of one system (``workloads.System`` or any object
    with the same fields).  potential="quadrature" integrates the local
    potential per cell by the Gauss rule (chfsi_op_build_quadrature)
    instead of collocating it at the nodes."""

    def __init__(self, ctx: Context, sys, potential: str = "nodal"):
        if potential not in ("nodal", "quadrature"):
            raise ValueError("potential must be 'nodal' or 'quadrature'")
        self.ctx = ctx
        lib = ctx.lib
        na = int(sys.pos.shape[0])
        self._keep = []

        def arr(x, n):
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))
            self._keep.append(a)
            return _dptr(a)

        s = _lib.System()
        s.L = float(sys.L)
        s.ncell = int(sys.ncell)
        s.p = int(sys.p)
        s.natoms = na
        s.has_proj = 1 if sys.has_proj else 0
        if na:
            s.pos = arr(sys.pos, 3 * na)
            s.Z = arr(sys.Z, na)
            s.s = arr(sys.s, na)
            if sys.has_proj:
                s.w = arr(sys.w, na)
                s.h_s = arr(sys.h_s, na)
                s.h_p = arr(sys.h_p, na)
        k = np.asarray(sys.k, dtype=np.float64)
        for i in range(3):
            s.k[i] = float(k[i])
        h = C.c_void_p()
        if not getattr(ctx, "h", None):
            raise ValueError("context is closed")
        build = lib.chfsi_op_build if potential == "nodal" else lib.chfsi_op_build_quadrature
        ctx.check(build(ctx.h, C.byref(s), C.byref(h)))
        self.h = h
        ctx._ops.add(self)
        self._keep.clear()
        M, E, npairs = C.c_int64(), C.c_int64(), C.c_int64()
        mc, npj, cp = C.c_int32(), C.c_int32(), C.c_int32()
        ctx.check(lib.chfsi_op_info(h, C.byref(M), C.byref(E), C.byref(mc), C.byref(npj), C.byref(npairs),
                                    C.byref(cp)))
        self.M, self.E, self.mcell = M.value, E.value, mc.value
        self.nproj, self.npairs, self.is_complex = npj.value, npairs.value, bool(cp.value)
        self.p = int(sys.p)
        self.ncell = int(sys.ncell)

    # -- tables -------------------------------------------------------------
    def tables(self):
        mc, M = self.mcell, self.M
        xyz = np.zeros((M, 3))
        cre = np.zeros((mc, mc))
        cim = np.zeros((mc, mc))
        vd = np.zeros(M)
        ds = np.zeros(M)
        self.ctx.check(self.ctx.lib.chfsi_op_tables(self.h, _dptr(xyz), _dptr(cre), _dptr(cim), _dptr(vd), _dptr(ds)))
        return {"xyz": xyz, "cell": cre + 1j * cim if self.is_complex else cre, "vdiag": vd, "dscale": ds}

    # -- steps of the method -----------------------------------------------
    def apply(self, X, Y, prec: Optional[int] = None):
        """Y = H~ X (device tensors, same storage type, same ld)."""
        if prec is None:
            prec = C128 if self.is_complex else F64
        ncols, ld = _ld_cols(X)
        ncols_y, ld_y = _ld_cols(Y)
        if ld_y != ld or ncols_y != ncols:
            raise ValueError("X and Y must have the same shape and ld")
        self.ctx.check(self.ctx.lib.chfsi_apply(self.h, _tptr(X), _tptr(Y), ncols, ld, int(prec)))

    def density(self, X, w, rho, points: int = RHO_NODES, accumulate: bool = False):
        """chfsi_density: rho (device float64; M values at the nodes, or
        E x (p+1)^3 at the Gauss points) (+)= sum_c w_c |M^-1/2 X_c|^2
        interpolated by the FE basis; X is the FP64 / complex128 block."""
        ncols, ld = _ld_cols(X)
        w = np.ascontiguousarray(w, dtype=np.float64)
        if w.size != ncols:
            raise ValueError("one weight per column")
        n_out = self.M if points == RHO_NODES else self.E * (self.p + 1) ** 3
        if rho.numel() != n_out:
            raise ValueError(f"rho must hold {n_out} values")
        self.ctx.check(self.ctx.lib.chfsi_density(self.h, _bptr(X), ncols, ld, _dptr(w), int(points),
                                                  int(bool(accumulate)), _tptr(rho)))

    def rayleigh_ritz_split(self, X, nfr: int, Psi_fr, mixed: bool = False):
        """chfsi_rayleigh_ritz_split: X (FP64 filtered block) becomes Psi_o;
        Psi_fr receives the nfr highest Ritz vectors; returns all N
        generalised eigenvalues."""
        ncols, ld = _ld_cols(X)
        nf, ldf = _ld_cols(Psi_fr)
        if nf != nfr:
            raise ValueError("Psi_fr must have nfr columns")
        th = np.zeros(ncols)
        self.ctx.check(self.ctx.lib.chfsi_rayleigh_ritz_split(self.h, _bptr(X), ncols, ld, int(nfr),
                                                              int(bool(mixed)), _dptr(th), _bptr(Psi_fr), ldf))
        return th

    def set_potential(self, V):
        """chfsi_op_set_potential: nodal local potential V (device float64, M)."""
        self.ctx.check(self.ctx.lib.chfsi_op_set_potential(self.h, _tptr(V)))

    def hartree(self, rho, vH, tol: float = 1e-10, maxit: int = 5000):
        """chfsi_hartree: vH <- Hartree potential of rho (device float64, M);
        returns (iterations, relative residual)."""
        it, rr = C.c_int32(), C.c_double()
        self.ctx.check(self.ctx.lib.chfsi_hartree(self.h, _tptr(rho), _tptr(vH), float(tol), int(maxit),
                                                  C.byref(it), C.byref(rr)), allow=(0, 1))
        return it.value, rr.value

    def scf(self, X, rho, nwanted: int, n_buf: int, n_electrons: float, kT: float, m: int = 20, block: int = 0,
            beta: float = 0.3, depth: int = 4, tol: float = 1e-8, maxit: int = 60, rr_mode: int = 2):
        """chfsi_scf: self-consistent loop; X (start block -> last basis) and
        rho (initial -> final density) are device tensors.  rr_mode: 0 full
        Rayleigh-Ritz, 1 spectrum splitting in FP64, 2 spectrum splitting with
        the mixed-precision blocks (default, the paper's form)."""
        ncols, ld = _ld_cols(X)
        if ncols != nwanted + n_buf:
            raise ValueError("X must have nwanted + n_buf columns")
        th = np.zeros(ncols)
        hist = np.zeros(maxit)
        mu, it = C.c_double(), C.c_int32()
        rc = self.ctx.check(self.ctx.lib.chfsi_scf(self.h, _tptr(X), ld, int(nwanted), int(n_buf), int(m), int(block),
                                                   int(rr_mode), float(n_electrons), float(kT), float(beta), int(depth), float(tol),
                                                   int(maxit), _tptr(rho), _dptr(th), C.byref(mu), _dptr(hist),
                                                   C.byref(it)), allow=(0, 1))
        return {"theta": th, "mu": mu.value, "iters": it.value, "residuals": hist[:it.value],
                "converged": rc == 0}

    def bounds(self, steps: int = 20, v0=None, seed: int = 0):
        b, lmin = C.c_double(), C.c_double()
        self.ctx.check(self.ctx.lib.chfsi_bounds(self.h, int(steps), _tptr(v0), C.c_uint64(seed), C.byref(b),
                                                 C.byref(lmin)))
        return b.value, lmin.value

    def filter(self, X, m: int, a: float, b: float, aL: float, prec: Optional[int] = None, block: int = 0):
        if prec is None:
            prec = C128 if self.is_complex else F64
        ncols, ld = _ld_cols(X)
        self.ctx.check(self.ctx.lib.chfsi_filter(self.h, _tptr(X), ncols, ld, int(m), float(a), float(b),
                                                 float(aL), int(prec), int(block)))

    def orthonormalize(self, X, want_L: bool = False):
        ncols, ld = _ld_cols(X)
        L = None
        ptr = C.POINTER(C.c_double)()
        if want_L:
            L = np.zeros((ncols, ncols), dtype=np.complex128 if self.is_complex else np.float64)
            ptr = L.ctypes.data_as(C.POINTER(C.c_double))
        self.ctx.check(self.ctx.lib.chfsi_orthonormalize(self.h, _tptr(X), ncols, ld, ptr))
        return L

    def rayleigh_ritz(self, X, want_resid: bool = True):
        ncols, ld = _ld_cols(X)
        th = np.zeros(ncols)
        r = np.zeros(ncols) if want_resid else None
        self.ctx.check(self.ctx.lib.chfsi_rayleigh_ritz(self.h, _tptr(X), ncols, ld, _dptr(th),
                                                        _dptr(r) if r is not None else C.POINTER(C.c_double)()))
        return th, r

    def solve(self, X, nwanted: int, m: int, block: int, n_buf: int = 0, fixed_passes: int = 0,
              tol: float = 0.0, max_passes: int = 100, filter_prec: Optional[int] = None,
              lanczos_steps: int = 20, b_upper: float = 0.0, lanczos_v0=None, seed: int = 0,
              prec_switch: bool = False, history: bool = False):
        """chfsi_solve.  With history=True, stats["history"] holds per-pass
        time_ms, max_resid, prec and theta (row 0: the initial Rayleigh-Ritz)."""
        if filter_prec is None:
            filter_prec = C128 if self.is_complex else F64
        ncols, ld = _ld_cols(X)
        if ncols != nwanted + n_buf:
            raise ValueError("X must have nwanted + n_buf columns")
        p = _lib.Params()
        p.nwanted, p.n_buf, p.m, p.block = nwanted, n_buf, m, block
        p.fixed_passes, p.max_passes, p.tol = fixed_passes, max_passes, tol
        p.filter_prec, p.lanczos_steps, p.b_upper = int(filter_prec), lanczos_steps, b_upper
        v0 = None
        if lanczos_v0 is not None:
            v0 = np.ascontiguousarray(lanczos_v0)
            if np.iscomplexobj(v0):
                v0 = v0.view(np.float64)
            v0 = np.ascontiguousarray(v0, dtype=np.float64)
            p.lanczos_v0 = _dptr(v0)
        p.seed = seed
        p.prec_switch = 1 if prec_switch else 0
        hist = _attach_history(p, ncols, fixed_passes, max_passes) if history else None
        th = np.zeros(ncols)
        r = np.zeros(ncols)
        st = _lib.Stats()
        rc = self.ctx.lib.chfsi_solve(self.h, C.byref(p), _tptr(X), ld, _dptr(th), _dptr(r), C.byref(st))
        self.ctx.check(rc, allow=(0, 1))
        stats = {f: getattr(st, f) for f, _ in _lib.Stats._fields_}
        stats["converged"] = rc == 0
        if hist is not None:
            stats["history"] = _trim_history(hist, stats["passes"])
        return th, r, stats

    def one_pass(self, X, nwanted: int, m: int, block: int, a: float, b: float, aL: float, n_buf: int = 0,
                 filter_prec: Optional[int] = None):
        """One ChFSI pass (filter, CholGS, Rayleigh-Ritz); returns (theta, resid)."""
        if filter_prec is None:
            filter_prec = C128 if self.is_complex else F64
        ncols, ld = _ld_cols(X)
        if ncols != nwanted + n_buf:
            raise ValueError("X must have nwanted + n_buf columns")
        p = _lib.Params()
        p.nwanted, p.n_buf, p.m, p.block, p.filter_prec = nwanted, n_buf, m, block, int(filter_prec)
        th = np.zeros(ncols)
        r = np.zeros(ncols)
        self.ctx.check(self.ctx.lib.chfsi_pass(self.h, C.byref(p), _tptr(X), ld, float(a), float(b), float(aL),
                                               _dptr(th), _dptr(r)))
        return th, r

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.chfsi_op_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Network:
    """The warm-start network (chfsi_mlp_*): device features in, device block out."""

    def __init__(self, ctx: Context, din: int = 32, hidden: int = 128, dout: int = 128, seed: int = 0):
        self.ctx = ctx
        h = C.c_void_p()
        ctx.check(ctx.lib.chfsi_mlp_create(ctx.h, int(din), int(hidden), int(dout), C.c_uint64(seed), C.byref(h)))
        self.h = h
        ctx._ops.add(self)
        a, b, c, n = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        ctx.check(ctx.lib.chfsi_mlp_info(h, C.byref(a), C.byref(b), C.byref(c), C.byref(n)))
        self.din, self.hidden, self.dout, self.nparams = a.value, b.value, c.value, n.value

    def params(self) -> np.ndarray:
        out = np.zeros(self.nparams, dtype=np.float32)
        self.ctx.check(self.ctx.lib.chfsi_mlp_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float)), 1))
        return out

    def set_params(self, vec) -> None:
        v = np.ascontiguousarray(vec, dtype=np.float32)
        if v.size != self.nparams:
            raise ValueError("wrong parameter count")
        self.ctx.check(self.ctx.lib.chfsi_mlp_params(self.h, v.ctypes.data_as(C.POINTER(C.c_float)), 0))

    def set_norm(self, mean, scale) -> None:
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(scale, dtype=np.float32)
        self.ctx.check(self.ctx.lib.chfsi_mlp_set_norm(self.h, m.ctypes.data_as(C.POINTER(C.c_float)),
                                                       s.ctypes.data_as(C.POINTER(C.c_float))))

    def forward(self, F, Y) -> None:
        self.ctx.check(self.ctx.lib.chfsi_mlp_forward(self.h, _tptr(F), F.shape[0], _tptr(Y)))

    def loss_grad(self, F, Q, want_grads: bool = True):
        loss = C.c_double()
        g = np.zeros(self.nparams, dtype=np.float32) if want_grads else None
        gp = g.ctypes.data_as(C.POINTER(C.c_float)) if want_grads else C.POINTER(C.c_float)()
        self.ctx.check(self.ctx.lib.chfsi_mlp_loss_grad(self.h, _tptr(F), F.shape[0], _tptr(Q), Q.shape[1],
                                                        C.byref(loss), gp))
        return loss.value, g

    def train_step(self, F, Q, lr: float = 1e-3) -> float:
        loss = C.c_double()
        self.ctx.check(self.ctx.lib.chfsi_mlp_train_step(self.h, _tptr(F), F.shape[0], _tptr(Q), Q.shape[1],
                                                         C.c_float(lr), C.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.chfsi_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def next_prec(prec: int, max_resid_history, b_upper: float) -> int:
    """chfsi_next_prec: filter precision for the next pass of a caller-driven
    solve, given max residuals after the initial Rayleigh-Ritz and each pass."""
    h = np.ascontiguousarray(max_resid_history, dtype=np.float64)
    return int(_lib.load().chfsi_next_prec(int(prec), _dptr(h), int(h.size - 1), float(b_upper)))


def fermi_level(theta, n_electrons: float, kT: float, weights=None):
    """chfsi_fermi_level: (mu, occupations) with 2 sum_i w_i f_i = n_electrons."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    if w is not None and w.size != th.size:
        raise ValueError("one weight per Ritz value")
    mu = C.c_double()
    occ = np.empty_like(th)
    rc = _lib.load().chfsi_fermi_level(_dptr(th), int(th.size), None if w is None else _dptr(w), float(n_electrons),
                                       float(kT), C.byref(mu), _dptr(occ))
    if rc != 0:
        raise ChfsiError(rc, "chfsi_fermi_level: need 0 < n_electrons < 2 sum(w), kT > 0, finite values")
    return mu.value, occ


def features(op: Operator, F) -> None:
    """F (device float32, M x 32) <- radial features of the operator's atoms."""
    op.ctx.check(op.ctx.lib.chfsi_features(op.h, _tptr(F)))


def initial_block(op: Operator, X, net: Optional[Network] = None, seed: int = 0) -> bool:
    """X (device float64, M x ld) <- warm start (or random); returns True if the fallback was used."""
    ncols, ld = _ld_cols(X)
    fb = C.c_int32()
    op.ctx.check(op.ctx.lib.chfsi_initial_block(op.h, net.h if net is not None else None, C.c_uint64(seed),
                                                _tptr(X), ncols, ld, C.byref(fb)))
    return bool(fb.value)
