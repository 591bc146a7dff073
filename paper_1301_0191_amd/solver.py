"""Python surface of the HIP library: a handle with the C ABI's calls.

PyTorch provides device memory and the stream; every numeric step runs in
libambddc.so (see include/ambddc.h for the semantics of each call).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _torch():
    import torch
    return torch


def _dev_ptr(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    return C.c_void_p(t.data_ptr())


def _initial(initial, face_averages):
    if face_averages:
        initial = "c+e+f"
    if initial not in _lib.INITIAL:
        raise ValueError(f"initial constraints must be one of {sorted(_lib.INITIAL)}")
    return _lib.INITIAL[initial]


def analyze(coords, elem_nodes, dirichlet, dof_per_node, elem_to_sub, face_averages=False,
            initial="c+e"):
    """Host-only level-1 structure counts and per-subdomain (n_I, n_Gamma)."""
    lib = _lib.load()
    co = np.ascontiguousarray(coords, dtype=np.float64)
    en = np.ascontiguousarray(elem_nodes, dtype=np.int32)
    di = np.ascontiguousarray(dirichlet, dtype=np.uint8)
    e2s = np.ascontiguousarray(elem_to_sub, dtype=np.int32)
    mesh = _lib.Mesh(co.shape[0], en.shape[0], dof_per_node, _ptr(co, C.c_double),
                     _ptr(en, C.c_int32), _ptr(di, C.c_uint8))
    dec = _lib.Decomp(2, _ptr(e2s, C.c_int32), None)
    out = _lib.Analysis()
    nsub = int(e2s.max()) + 1
    sizes = np.zeros(2 * nsub, dtype=np.int32)
    _lib.check(lib.ambddc_analyze(C.byref(mesh), C.byref(dec), _initial(initial, face_averages),
                                  C.byref(out), sizes.ctypes.data_as(C.c_void_p), nsub))
    d = {f: getattr(out, f) for f, _ in _lib.Analysis._fields_}
    d["sub_sizes"] = sizes.reshape(nsub, 2)
    return d


@dataclass
class SolveResult:
    x: object
    iterations: list
    cond: list
    true_residual: list = None   # ||f - K x|| / ||f|| per column, recomputed after PCG


class Handle:
    """One problem: mesh + decomposition (create), coefficients (setup), solves."""

    def __init__(self, coords, elem_nodes, dirichlet, dof_per_node, elem_to_sub, parents=(),
                 levels=2, tau=10.0, nev_max=10, lobpcg_maxit=100, lobpcg_block=16,
                 lobpcg_tol=1e-7, face_averages=False, seed=12345, stream=None, precision=0,
                 initial="c+e", keep_edges=False, fixed_per_face=0):
        """precision 0: FP64 throughout; 1: the PCG preconditioner's dense
        subdomain operators are kept in FP32 (widened to FP64 on load),
        everything else in FP64; 2: as 1, and the pair LOBPCG runs its
        operator products in FP32 on MFMA until each pair's residual reaches
        1e-5 (or stalls), then polishes in FP64.  initial: "c+e" (default), "c+e+f" (or
        face_averages=True) or "c"; keep_edges: adaptive rows keep their
        entries on shared edges and corners; fixed_per_face = k > 0: k
        eigenvector constraints per face regardless of tau ("3eigv": 3)."""
        if precision not in (0, 1, 2):
            raise ValueError("precision must be 0, 1 or 2")
        lib = _lib.load()
        self._lib = lib
        self._coords = np.ascontiguousarray(coords, dtype=np.float64)
        self._en = np.ascontiguousarray(elem_nodes, dtype=np.int32)
        self._dir = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        self._e2s = np.ascontiguousarray(elem_to_sub, dtype=np.int32)
        self._par = [np.ascontiguousarray(p, dtype=np.int32) for p in parents]
        mesh = _lib.Mesh(self._coords.shape[0], self._en.shape[0], dof_per_node,
                         _ptr(self._coords, C.c_double), _ptr(self._en, C.c_int32),
                         _ptr(self._dir, C.c_uint8))
        par_arr = (C.POINTER(C.c_int32) * max(1, len(self._par)))(
            *[_ptr(p, C.c_int32) for p in self._par])
        dec = _lib.Decomp(levels, _ptr(self._e2s, C.c_int32), par_arr)
        opt = _lib.Options()
        lib.ambddc_default_options(C.byref(opt))
        opt.tau = float(tau)
        opt.nev_max = int(nev_max)
        opt.lobpcg_maxit = int(lobpcg_maxit)
        opt.lobpcg_block = int(lobpcg_block)
        opt.lobpcg_tol = float(lobpcg_tol)
        opt.initial_constraints = _initial(initial, face_averages)
        opt.keep_edges = int(bool(keep_edges))
        opt.fixed_per_face = int(fixed_per_face)
        opt.precision = int(precision)
        opt.seed = int(seed)
        if stream is None:
            torch = _torch()
            stream = torch.cuda.current_stream().cuda_stream
        opt.stream = C.c_void_p(stream)
        h = C.c_void_p()
        _lib.check(lib.ambddc_create(C.byref(mesh), C.byref(dec), C.byref(opt), C.byref(h)))
        self._h = h
        self.setup_count = 0   # set-up calls on this handle (numeric state version)
        self.dof_per_node = dof_per_node
        self.precision = int(precision)
        self.n_elems = int(self._en.shape[0])
        self.n_free = int(np.count_nonzero(self._dir == 0))

    @classmethod
    def from_problem(cls, prob, **kw):
        kw.setdefault("tau", prob.tau)
        kw.setdefault("nev_max", prob.nev_max)
        return cls(prob.coords, prob.elem_nodes, prob.dirichlet, prob.dof_per_node,
                   prob.elem_to_sub, prob.parents, levels=prob.levels, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.ambddc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- numeric calls --------------------------------------------------
    def setup(self, coeff, nu=None, check=True):
        """coeff, nu: float64 GPU tensors of length n_elems."""
        self.setup_count += 1
        code = self._lib.ambddc_setup(self._h, _dev_ptr(coeff), None if nu is None else _dev_ptr(nu))
        if check:
            _lib.check(code)
        return code

    def solve(self, rhs, rtol=1e-10, maxit=1000, x=None, raise_on_noconv=True):
        """rhs: float64 GPU tensor (n_free,) or (nrhs, n_free) (row r = column r)."""
        torch = _torch()
        r2 = rhs if rhs.dim() == 2 else rhs.view(1, -1)
        nrhs = r2.shape[0]
        if x is None:
            x = torch.empty_like(r2)
        its = (C.c_int32 * nrhs)()
        cond = (C.c_double * nrhs)()
        code = self._lib.ambddc_solve(self._h, _dev_ptr(r2), nrhs, float(rtol), int(maxit),
                                      _dev_ptr(x), its, cond)
        if code != 0 and (raise_on_noconv or code != 4):
            _lib.check(code)
        xs = x if rhs.dim() == 2 else x.view(-1)
        res = (C.c_double * nrhs)()
        tr = None
        if self._lib.ambddc_last_residual(self._h, nrhs, res) == 0:
            tr = list(res)
        return SolveResult(xs, list(its), list(cond), tr)

    def solve_noalloc(self, rhs, x, rtol=1e-10, maxit=1000, raise_on_noconv=True):
        """ambddc_solve_noalloc: rhs and x are float64 GPU tensors of the same
        shape, (n_free,) or (nrhs, n_free), nrhs <= 3; the library allocates
        no device memory in this call."""
        r2 = rhs if rhs.dim() == 2 else rhs.view(1, -1)
        x2 = x if x.dim() == 2 else x.view(1, -1)
        if x2.shape != r2.shape:
            raise ValueError("x must have the shape of rhs")
        nrhs = r2.shape[0]
        its = (C.c_int32 * nrhs)()
        cond = (C.c_double * nrhs)()
        code = self._lib.ambddc_solve_noalloc(self._h, _dev_ptr(r2), nrhs, float(rtol),
                                              int(maxit), _dev_ptr(x2), its, cond)
        if code != 0 and (raise_on_noconv or code != 4):
            _lib.check(code)
        res = (C.c_double * nrhs)()
        tr = None
        if self._lib.ambddc_last_residual(self._h, nrhs, res) == 0:
            tr = list(res)
        return SolveResult(x, list(its), list(cond), tr)

    def setup_log10(self, theta, nu=None, check=True):
        """Set-up with coefficients 10^theta computed on the device."""
        self.setup_count += 1
        code = self._lib.ambddc_setup_log10(self._h, _dev_ptr(theta),
                                            None if nu is None else _dev_ptr(nu))
        if check:
            _lib.check(code)
        return code

    def misfit(self, X, Xobs, R=None):
        """R = X - Xobs on the device and J = 1/2 ||R||_F^2; returns (J, R)."""
        torch = _torch()
        X2 = X if X.dim() == 2 else X.view(1, -1)
        O2 = Xobs if Xobs.dim() == 2 else Xobs.view(1, -1)
        if R is None:
            R = torch.empty_like(X2)
        J = C.c_double()
        _lib.check(self._lib.ambddc_misfit(self._h, _dev_ptr(X2), _dev_ptr(O2), X2.shape[0],
                                           _dev_ptr(R), C.byref(J)))
        return J.value, R

    def element_gradient(self, X, Lam):
        torch = _torch()
        X2 = X if X.dim() == 2 else X.view(1, -1)
        L2 = Lam if Lam.dim() == 2 else Lam.view(1, -1)
        g = torch.empty(self.n_elems, dtype=torch.float64, device=X.device)
        _lib.check(self._lib.ambddc_element_gradient(self._h, _dev_ptr(X2), _dev_ptr(L2),
                                                     X2.shape[0], _dev_ptr(g)))
        return g

    # --- introspection --------------------------------------------------
    def stats(self):
        s = _lib.Stats()
        _lib.check(self._lib.ambddc_get_stats(self._h, C.byref(s)))
        L = s.levels
        return dict(levels=L, n_free=s.n_free, n_sub=list(s.n_sub[:L]),
                    n_pairs=list(s.n_pairs[:L]), n_coarse=list(s.n_coarse[:L]),
                    n_adaptive=list(s.n_adaptive[:L]), lobpcg_iters=list(s.lobpcg_iters[:L]),
                    lobpcg_iters_fp32=list(s.lobpcg_iters_fp32[:L]),
                    n_unconverged=list(s.n_unconverged[:L]),
                    omega_tilde=list(s.omega_tilde[:L]), t_phase=list(s.t_phase[:8]),
                    pcg_replacements=s.pcg_replacements, pcg_stalled=s.pcg_stalled)

    def level_info(self, level):
        a = [C.c_int32() for _ in range(4)]
        _lib.check(self._lib.ambddc_level_info(self._h, level, *[C.byref(x) for x in a]))
        return dict(n_dof=a[0].value, n_sub=a[1].value, n_pairs=a[2].value,
                    n_coarse=a[3].value)

    def sub_dofs(self, level, sub):
        nI, nG = C.c_int32(), C.c_int32()
        _lib.check(self._lib.ambddc_sub_dofs(self._h, level, sub, None, C.byref(nI),
                                             C.byref(nG)))
        d = np.empty(nI.value + nG.value, dtype=np.int32)
        _lib.check(self._lib.ambddc_sub_dofs(self._h, level, sub, d.ctypes.data_as(C.c_void_p),
                                             C.byref(nI), C.byref(nG)))
        return d, nI.value, nG.value

    def schur(self, level, sub):
        _, nI, nG = self.sub_dofs(level, sub)
        S = np.empty((nG, nG), dtype=np.float64, order="F")
        _lib.check(self._lib.ambddc_get_schur(self._h, level, sub, S.ctypes.data_as(C.c_void_p)))
        return S

    def pair_info(self, level, pair):
        s, t, nf = C.c_int32(), C.c_int32(), C.c_int32()
        _lib.check(self._lib.ambddc_pair_info(self._h, level, pair, C.byref(s), C.byref(t),
                                              C.byref(nf)))
        return s.value, t.value, nf.value

    def pair_result(self, level, pair):
        m = C.c_int32()
        _lib.check(self._lib.ambddc_get_pair_result(self._h, level, pair, 0, C.byref(m), None,
                                                    None, None, None, None, None))
        lam = np.zeros(m.value, dtype=np.float64)
        res = np.zeros(m.value, dtype=np.float64)
        k, it, cv = C.c_int32(), C.c_int32(), C.c_int32()
        ln = C.c_double()
        _lib.check(self._lib.ambddc_get_pair_result(self._h, level, pair, m.value, None,
                                                    lam.ctypes.data_as(C.c_void_p),
                                                    res.ctypes.data_as(C.c_void_p), C.byref(k),
                                                    C.byref(ln), C.byref(it), C.byref(cv)))
        return dict(lam=lam, resid=res, k=k.value, lam_next=ln.value, iters=it.value,
                    converged=bool(cv.value))

    def face_constraints(self, level, pair, k):
        _, _, nf = self.pair_info(level, pair)
        rows = np.zeros((max(k, 0), nf), dtype=np.float64)
        fd = np.zeros(nf, dtype=np.int32)
        _lib.check(self._lib.ambddc_get_face_constraints(
            self._h, level, pair, rows.ctypes.data_as(C.c_void_p), fd.ctypes.data_as(C.c_void_p)))
        return rows, fd

    def coarse_element(self, level, sub):
        nc = C.c_int32()
        _lib.check(self._lib.ambddc_get_coarse_element(self._h, level, sub, None, C.byref(nc)))
        K = np.zeros((nc.value, nc.value), dtype=np.float64, order="F")
        if nc.value:
            _lib.check(self._lib.ambddc_get_coarse_element(
                self._h, level, sub, K.ctypes.data_as(C.c_void_p), C.byref(nc)))
        return K

    def top_coarse(self):
        n = C.c_int32()
        _lib.check(self._lib.ambddc_get_top_coarse(self._h, None, C.byref(n)))
        K = np.zeros((n.value, n.value), dtype=np.float64, order="F")
        if n.value:
            _lib.check(self._lib.ambddc_get_top_coarse(self._h, K.ctypes.data_as(C.c_void_p),
                                                       C.byref(n)))
        return K

    # ---- PCG iteration graphs ----
    def set_graphs(self, on):
        """Replay PCG iterations as HIP graphs (ambddc_set_graphs)."""
        _lib.check(self._lib.ambddc_set_graphs(self._h, 1 if on else 0))

    # ---- kernel timing ----
    def timing_enable(self, classes):
        """Time the listed kernel classes (list or comma-separated string)
        with HIP events on the handle's stream; None switches timing off."""
        if classes is None:
            arg = None
        else:
            arg = (",".join(classes) if not isinstance(classes, str) else classes).encode()
        _lib.check(self._lib.ambddc_timing_enable(self._h, arg))

    def timing_read(self, cls):
        """{'launches', 'ms', 'flops', 'bytes'} summed since timing_enable."""
        n = C.c_int32()
        ms, fl, by = C.c_double(), C.c_double(), C.c_double()
        _lib.check(self._lib.ambddc_timing_read(self._h, cls.encode(), C.byref(n), C.byref(ms),
                                                C.byref(fl), C.byref(by)))
        return dict(launches=n.value, ms=ms.value, flops=fl.value, bytes=by.value)
