"""Plain FP64 CPU oracle for the non-negative diffusion QP (arXiv:1506.08435).

TEST INFRASTRUCTURE ONLY: imported by `tests/`, by `__graft_entry__.smoke()`
and by the CPU-baseline leg of `bench.py`, never by the product package.  It
shares no code with the HIP library.

* `assemble`      P1 stiffness / mass / load, Dirichlet nodes eliminated,
                  non-zero Dirichlet values lifted into the load
                  (Sec. 2.1.2-2.1.3; capacity matrix Sec. 2.2.2)  [oracle.c]
* `solve`         unique minimiser of 1/2 c.Kc - c.F s.t. lo <= c <= hi
                  (Sec. 2.1.3, eq. non-negative: [0, inf); Sec. 2.2.2 and
                  the DMP Remark of Sec. 5: [c_min, c_max])        [oracle.c]
* `galerkin`      unconstrained K c = F by Jacobi-PCG (Sec. 2.1.2) [oracle.c]
* `kkt`           KKT certificate of a candidate c               [oracle.c]
* `transient_step` one backward-Euler QP (Sec. 2.2.2)             [oracle.c]
* `brute.brute_force` exhaustive active-set enumeration, N <= 12   [brute.py]

The C part is compiled by `oracle/build.py` (gcc, no fast-math).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import time
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class OrStats(ctypes.Structure):
    _fields_ = [("r", ctypes.c_double), ("outer", ctypes.c_int64), ("gp_steps", ctypes.c_int64),
                ("cg_its", ctypes.c_int64), ("face_its", ctypes.c_int64),
                ("polishes", ctypes.c_int64), ("certified", ctypes.c_int64),
                ("floor", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.or_assemble.restype = ctypes.c_void_p
    lib.or_assemble.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _f64p, _i32p, _f64p,
                                ctypes.c_int64, _f64p, _f64p, _u8p, _f64p, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_int)]
    lib.or_free.argtypes = [ctypes.c_void_p]
    lib.or_problem_sizes.argtypes = [ctypes.c_void_p, _i64p, _i64p]
    lib.or_problem_export.argtypes = [ctypes.c_void_p, _i64p, _i32p, _f64p, _f64p, _f64p, _i64p]
    lib.or_spmv.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _f64p]
    lib.or_kkt.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, ctypes.c_double,
                           ctypes.c_double, _f64p, _f64p]
    lib.or_set_progress.argtypes = [ctypes.c_double]
    lib.or_solve.restype = ctypes.c_int
    lib.or_solve.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, ctypes.c_int64, _f64p,
                             ctypes.POINTER(OrStats)]
    lib.or_galerkin.restype = ctypes.c_int64
    lib.or_galerkin.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, ctypes.c_double, _f64p]
    lib.or_transient_step.restype = ctypes.c_int
    lib.or_transient_step.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, ctypes.c_double,
                                      _f64p, _f64p, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int64, _f64p,
                                      ctypes.POINTER(OrStats)]
    lib.or_transient_system.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p,
                                        ctypes.c_double, _f64p, _f64p, _f64p, _f64p]
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclasses.dataclass
class System:
    """Assembled free-DOF system: CSR (int64 rowptr, int32 col) + values."""
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    K: np.ndarray
    M: Optional[np.ndarray]
    F: np.ndarray
    dof: np.ndarray   # node -> free DOF index or -1

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    def to_scipy(self, which: str = "K"):
        import scipy.sparse as sp
        vals = self.K if which == "K" else self.M
        return sp.csr_matrix((vals, self.col, self.rowptr), shape=(self.n, self.n))


def assemble(problem, with_mass: bool = False) -> System:
    """Assemble from a problem object exposing dim, coords, elems, D, kscale,
    f_elem and dirichlet arrays (and optionally dirichlet_values: the value of
    c at each Dirichlet node, lifted into F)."""
    lib = _load()
    dim = int(problem.dim)
    coords = np.ascontiguousarray(problem.coords, dtype=np.float64)
    elems = np.ascontiguousarray(problem.elems, dtype=np.int32)
    D = np.ascontiguousarray(problem.D, dtype=np.float64)
    nD = D.size // (dim * dim)
    ks = None if problem.kscale is None else np.ascontiguousarray(problem.kscale, dtype=np.float64)
    f = np.ascontiguousarray(problem.f_elem, dtype=np.float64)
    dmask = np.ascontiguousarray(problem.dirichlet, dtype=np.uint8)
    dv = getattr(problem, "dirichlet_values", None)
    dv = None if dv is None else np.ascontiguousarray(dv, dtype=np.float64)
    st = ctypes.c_int(0)
    h = lib.or_assemble(dim, coords.shape[0], elems.shape[0], _p(coords, ctypes.c_double),
                        _p(elems, ctypes.c_int32), _p(D, ctypes.c_double), nD,
                        None if ks is None else _p(ks, ctypes.c_double), _p(f, ctypes.c_double),
                        _p(dmask, ctypes.c_uint8), None if dv is None else _p(dv, ctypes.c_double),
                        int(with_mass), ctypes.byref(st))
    if not h:
        raise RuntimeError(f"oracle assembly failed (status {st.value})")
    try:
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        lib.or_problem_sizes(h, ctypes.byref(n), ctypes.byref(nnz))
        rowptr = np.zeros(n.value + 1, dtype=np.int64)
        col = np.zeros(max(nnz.value, 1), dtype=np.int32)
        K = np.zeros(max(nnz.value, 1))
        M = np.zeros(max(nnz.value, 1)) if with_mass else None
        F = np.zeros(max(n.value, 1))
        dof = np.zeros(coords.shape[0], dtype=np.int64)
        lib.or_problem_export(h, _p(rowptr, ctypes.c_int64), _p(col, ctypes.c_int32),
                              _p(K, ctypes.c_double),
                              None if M is None else _p(M, ctypes.c_double),
                              _p(F, ctypes.c_double), _p(dof, ctypes.c_int64))
    finally:
        lib.or_free(h)
    m = nnz.value
    return System(n=n.value, rowptr=rowptr, col=col[:m], K=K[:m],
                  M=None if M is None else M[:m], F=F[:n.value], dof=dof)


def spmv(sysm: System, x: np.ndarray, vals: Optional[np.ndarray] = None) -> np.ndarray:
    lib = _load()
    v = sysm.K if vals is None else np.ascontiguousarray(vals, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(max(sysm.n, 1))
    lib.or_spmv(sysm.n, _p(sysm.rowptr, ctypes.c_int64), _p(sysm.col, ctypes.c_int32),
                _p(v, ctypes.c_double), _p(x, ctypes.c_double), _p(y, ctypes.c_double))
    return y[:sysm.n]


@dataclasses.dataclass
class KKT:
    r: float          # ||pg||_2 / ||F||_2
    nat_inf: float    # ||c - P(c - g)||_inf (= ||min(c, g)||_inf for [0, inf))
    min_c: float
    comp_inf: float   # max min(c_i - lo, hi - c_i) |g_i|
    normF: float
    nonfinite: int
    min_g_active: float   # min g over {c == lo}
    n_zero: int           # #{c == lo}
    max_c: float = 0.0
    max_g_upper: float = -np.inf   # max g over {c == hi}
    n_upper: int = 0               # #{c == hi}


def kkt(sysm: System, c: np.ndarray, F: Optional[np.ndarray] = None,
        vals: Optional[np.ndarray] = None, lo: float = 0.0, hi: float = np.inf) -> KKT:
    lib = _load()
    v = sysm.K if vals is None else np.ascontiguousarray(vals, dtype=np.float64)
    F = sysm.F if F is None else np.ascontiguousarray(F, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(11)
    lib.or_kkt(sysm.n, _p(sysm.rowptr, ctypes.c_int64), _p(sysm.col, ctypes.c_int32),
               _p(v, ctypes.c_double), _p(F, ctypes.c_double), float(lo), float(hi),
               _p(c, ctypes.c_double), _p(out, ctypes.c_double))
    return KKT(r=out[0], nat_inf=out[1], min_c=out[2], comp_inf=out[3], normF=out[4],
               nonfinite=int(out[5]), min_g_active=out[6], n_zero=int(out[7]), max_c=out[8],
               max_g_upper=out[9], n_upper=int(out[10]))


@dataclasses.dataclass
class SolveResult:
    c: np.ndarray
    status: int
    r: float
    outer: int
    gp_steps: int
    cg_its: int
    face_its: int
    polishes: int
    certified: bool
    seconds: float
    floor: float = 0.0


def solve(sysm: System, tol: float = 1e-12, c0: Optional[np.ndarray] = None,
          F: Optional[np.ndarray] = None, vals: Optional[np.ndarray] = None,
          max_outer: int = 20000, lo: float = 0.0, hi: float = np.inf) -> SolveResult:
    """Minimise 1/2 c.Kc - c.F over lo <= c <= hi to ||pg||/||F|| <= tol,
    finishing with a face solve and a KKT check."""
    lib = _load()
    v = sysm.K if vals is None else np.ascontiguousarray(vals, dtype=np.float64)
    F = sysm.F if F is None else np.ascontiguousarray(F, dtype=np.float64)
    c = np.zeros(max(sysm.n, 1)) if c0 is None else np.array(c0, dtype=np.float64, copy=True)
    st = OrStats()
    t0 = time.perf_counter()
    rc = lib.or_solve(sysm.n, _p(sysm.rowptr, ctypes.c_int64), _p(sysm.col, ctypes.c_int32),
                      _p(v, ctypes.c_double), _p(F, ctypes.c_double), float(lo), float(hi), tol,
                      max_outer, _p(c, ctypes.c_double), ctypes.byref(st))
    dt = time.perf_counter() - t0
    return SolveResult(c=c[:sysm.n], status=rc, r=st.r, outer=st.outer, gp_steps=st.gp_steps,
                       cg_its=st.cg_its, face_its=st.face_its, polishes=st.polishes,
                       certified=bool(st.certified), seconds=dt, floor=st.floor)


def galerkin(sysm: System, rtol: float = 1e-13) -> np.ndarray:
    """Unconstrained Galerkin solution K c = F (Jacobi-PCG)."""
    lib = _load()
    c = np.zeros(max(sysm.n, 1))
    lib.or_galerkin(sysm.n, _p(sysm.rowptr, ctypes.c_int64), _p(sysm.col, ctypes.c_int32),
                    _p(sysm.K, ctypes.c_double), _p(sysm.F, ctypes.c_double), rtol,
                    _p(c, ctypes.c_double))
    return c[:sysm.n]


def transient_system(sysm: System, dt: float, cn: np.ndarray):
    """(K~ values, f~) of one backward-Euler step."""
    lib = _load()
    Kt = np.zeros(max(sysm.nnz, 1))
    ft = np.zeros(max(sysm.n, 1))
    cn = np.ascontiguousarray(cn, dtype=np.float64)
    lib.or_transient_system(sysm.n, _p(sysm.rowptr, ctypes.c_int64), _p(sysm.col, ctypes.c_int32),
                            _p(sysm.K, ctypes.c_double), _p(sysm.M, ctypes.c_double), dt,
                            _p(sysm.F, ctypes.c_double), _p(cn, ctypes.c_double),
                            _p(Kt, ctypes.c_double), _p(ft, ctypes.c_double))
    return Kt[:sysm.nnz], ft[:sysm.n]


def transient_step(sysm: System, dt: float, cn: np.ndarray, tol: float = 1e-12,
                   max_outer: int = 20000, lo: float = 0.0, hi: float = np.inf) -> SolveResult:
    lib = _load()
    cn = np.ascontiguousarray(cn, dtype=np.float64)
    c = np.zeros(max(sysm.n, 1))
    st = OrStats()
    t0 = time.perf_counter()
    rc = lib.or_transient_step(sysm.n, _p(sysm.rowptr, ctypes.c_int64),
                               _p(sysm.col, ctypes.c_int32), _p(sysm.K, ctypes.c_double),
                               _p(sysm.M, ctypes.c_double), dt, _p(sysm.F, ctypes.c_double),
                               _p(cn, ctypes.c_double), float(lo), float(hi), tol, max_outer,
                               _p(c, ctypes.c_double), ctypes.byref(st))
    dt_s = time.perf_counter() - t0
    return SolveResult(c=c[:sysm.n], status=rc, r=st.r, outer=st.outer, gp_steps=st.gp_steps,
                       cg_its=st.cg_its, face_its=st.face_its, polishes=st.polishes,
                       certified=bool(st.certified), seconds=dt_s, floor=st.floor)


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(t: int) -> None:
    _load().or_set_num_threads(int(t))


def set_progress(seconds: float) -> None:
    """Progress lines on stderr, at most one every `seconds` (0: none)."""
    _load().or_set_progress(float(seconds))


def nondegenerate_masks(c_ref: np.ndarray, g_ref: np.ndarray, F: np.ndarray, rel: float = 1e-8,
                        lo: float = 0.0, hi: float = np.inf):
    """Nodes whose status the oracle fixes unambiguously: free if c is more
    than rel*||c||_inf inside both bounds, strictly active if c is at a bound
    with a gradient of the binding sign larger than rel*||F||_inf (returned
    together: at lo, or at hi)."""
    cmax = float(np.max(np.abs(c_ref))) if c_ref.size else 0.0
    fmax = float(np.max(np.abs(F))) if F.size else 0.0
    free = (c_ref > lo + rel * cmax) & (c_ref < hi - rel * cmax)
    strict = ((c_ref == lo) & (g_ref > rel * fmax)) | ((c_ref == hi) & (g_ref < -rel * fmax))
    return free, strict
