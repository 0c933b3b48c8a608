"""Python binding of the C ABI in include/nnqp.h (ctypes over libnnqp.so).

Argument marshalling only: every step of assembly and solve runs in the HIP
library.  Device buffers are torch tensors on the context's device; streams
are torch streams.  Function names follow the C entry points without the
`nn_` prefix.  There is no fallback: if libnnqp.so is missing or no GPU is
present, `Context()` raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnnqp.so")

NN_OK, NN_EINVAL, NN_ENONFINITE, NN_ENOTSPD, NN_EMAXIT, NN_EOOM, NN_EHIP, NN_EBUDGET = range(8)
NN_FP64, NN_MIXED = 0, 1
NN_TRON, NN_BLMVM = 0, 1
NN_KCLASSES = 5
NN_PROF_ALL = 0x1F
KCLASS_NAMES = ("cg_spmv", "cg_update", "grad", "trial", "other")
STATUS_NAMES = {0: "NN_OK", 1: "NN_EINVAL", 2: "NN_ENONFINITE", 3: "NN_ENOTSPD", 4: "NN_EMAXIT",
                5: "NN_EOOM", 6: "NN_EHIP", 7: "NN_EBUDGET"}

# exported symbols declared in include/nnqp.h (checked by the ABI test)
SYMBOLS = ("nn_create", "nn_create_ex", "nn_destroy", "nn_last_error", "nn_default_opts", "nn_assemble",
           "nn_matrix_from_csr", "nn_matrix_info", "nn_matrix_export", "nn_matrix_bytes",
           "nn_matrix_free", "nn_matvec", "nn_solve_nonneg", "nn_solve_nonneg_noalloc",
           "nn_solve_galerkin", "nn_step_transient",
           "nn_solve_batch", "nn_step_transient_batch", "nn_set_profiling", "nn_set_profiling_sample", "nn_kernel_times")


# device memory hooks of nn_create_ex: alloc(bytes, user) -> pointer or NULL,
# free_(pointer, user)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class NnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_nodes", ctypes.c_int64), ("n_elems", ctypes.c_int64),
                ("coords", ctypes.c_void_p), ("elems", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("max_cg", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("c0_mode", ctypes.c_int32),
                ("c0_value", ctypes.c_double), ("delta0", ctypes.c_double),
                ("cg_chunk", ctypes.c_int32), ("verbose", ctypes.c_int32),
                ("lower", ctypes.c_double), ("upper", ctypes.c_double),
                ("method", ctypes.c_int32), ("lmm_vectors", ctypes.c_int32),
                ("max_lm_its", ctypes.c_int32), ("precond_degree", ctypes.c_int32),
                ("subspace", ctypes.c_int32), ("engine", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("kkt_rel", ctypes.c_double), ("kkt_nat_inf", ctypes.c_double),
                ("min_c", ctypes.c_double), ("norm_f", ctypes.c_double),
                ("outer_its", ctypes.c_int32), ("cg_its", ctypes.c_int32),
                ("spmvs", ctypes.c_int32), ("n_active", ctypes.c_int32),
                ("cauchy_trials", ctypes.c_int32), ("search_trials", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("status", ctypes.c_int32),
                ("bytes_moved", ctypes.c_double), ("seconds", ctypes.c_double),
                ("max_c", ctypes.c_double), ("n_negative", ctypes.c_int32),
                ("subspace_its", ctypes.c_int32), ("radius_stops", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libnnqp.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime under the same soname as /opt/rocm's; it
    # must be loaded first so that this library binds to the runtime that owns
    # torch's device memory and streams (one runtime per process).
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or paper_1506_08435_amd/build.py)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "nn_create": (i32, [P(vp), ctypes.c_int, vp]),
        "nn_create_ex": (i32, [P(vp), ctypes.c_int, vp, ALLOC_FN, FREE_FN, vp]),
        "nn_destroy": (None, [vp]),
        "nn_last_error": (ctypes.c_char_p, [vp]),
        "nn_default_opts": (i32, [P(Opts)]),
        "nn_assemble": (i32, [vp, P(Mesh), vp, i64, vp, vp, vp, vp, ctypes.c_int, P(vp), vp, vp]),
        "nn_matrix_from_csr": (i32, [vp, i64, vp, vp, vp, vp, P(vp)]),
        "nn_matrix_info": (i32, [vp, P(i64), P(i64), P(ctypes.c_int)]),
        "nn_matrix_export": (i32, [vp, vp, vp, vp, vp, vp]),
        "nn_matrix_bytes": (i32, [vp, ctypes.c_int, P(ctypes.c_size_t)]),
        "nn_matrix_free": (None, [vp, vp]),
        "nn_matvec": (i32, [vp, vp, ctypes.c_int, vp, vp]),
        "nn_solve_nonneg": (i32, [vp, vp, vp, P(Opts), vp, vp, P(Stats)]),
        "nn_solve_nonneg_noalloc": (i32, [vp, vp, vp, P(Opts), vp, vp, P(Stats)]),
        "nn_solve_galerkin": (i32, [vp, vp, vp, P(Opts), vp, P(Stats)]),
        "nn_step_transient": (i32, [vp, vp, dbl, vp, P(Opts), vp, vp, P(Stats)]),
        "nn_solve_batch": (i32, [vp, i32, P(vp), P(vp), P(Opts), P(vp), P(vp), P(Stats)]),
        "nn_step_transient_batch": (i32, [vp, i32, P(vp), dbl, P(vp), P(Opts), P(vp), P(vp),
                                          P(Stats)]),
        "nn_set_profiling": (i32, [vp, ctypes.c_int]),
        "nn_set_profiling_sample": (i32, [vp, i32]),
        "nn_kernel_times": (i32, [vp, vp, vp, vp, vp, ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def default_opts(**kw) -> Opts:
    o = Opts()
    load_library().nn_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    return a.data_ptr()


@dataclasses.dataclass
class Matrix:
    ctx: "Context"
    handle: int
    n: int
    nnz: int
    has_mass: bool

    def bytes(self, precision: int = NN_FP64) -> int:
        """Device bytes of the matrix and one solve's work vectors (nn_matrix_bytes)."""
        return self.ctx.matrix_bytes(self, precision)

    def free(self):
        if self.handle:
            self.ctx.lib.nn_matrix_free(self.ctx.handle, self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """One device + one stream (torch's current stream unless given).

    allocator: None, the library takes device memory with hipMalloc; "torch",
    every device buffer of the context and of the matrices it creates comes
    from torch's caching allocator on this context's stream; or a pair of
    callables (alloc(nbytes) -> device pointer as int, or None; free(ptr)).
    The last two go through nn_create_ex.  Matrices keep a reference to their
    context, so the hooks outlive them."""

    def __init__(self, device: int = 0, stream=None, allocator=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the nnqp library needs an MI355X")
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(self.stream.cuda_stream)
        self._hooks = None
        if allocator is None:
            st = self.lib.nn_create(ctypes.byref(h), device, sp)
        else:
            if allocator == "torch":
                dev, strm = device, self.stream
                alloc_py = lambda nbytes: torch.cuda.caching_allocator_alloc(nbytes, dev, strm)
                free_py = torch.cuda.caching_allocator_delete
            elif isinstance(allocator, tuple) and len(allocator) == 2 and all(map(callable, allocator)):
                alloc_py, free_py = allocator
            else:
                raise ValueError(f"allocator must be None, 'torch' or (alloc, free), not {allocator!r}")

            def _alloc(nbytes, _user):
                try:
                    return alloc_py(int(nbytes)) or None
                except Exception:   # out of memory: the library reports NN_EOOM
                    return None

            def _free(ptr, _user):
                free_py(ptr)

            self._hooks = (ALLOC_FN(_alloc), FREE_FN(_free))
            st = self.lib.nn_create_ex(ctypes.byref(h), device, sp, self._hooks[0], self._hooks[1], None)
        if st != NN_OK:
            raise NnError(st, "nn_create failed")
        self.handle = h.value

    def close(self):
        if getattr(self, "handle", None):
            self.lib.nn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self.lib.nn_last_error(self.handle).decode()

    def _check(self, st: int, what: str, allow=(NN_OK,)):
        if st not in allow:
            raise NnError(st, f"{what}: {self.last_error()}")
        return st

    # ---------------------------------------------------------------- matrices
    def assemble(self, problem, with_mass: bool = False):
        """(Matrix, F [n] device float64, dof_of_node [n_nodes] int64 numpy)."""
        t = self.torch
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
        n = int((dmask == 0).sum())
        mesh = Mesh(dim, coords.shape[0], elems.shape[0], _ptr(coords), _ptr(elems))
        F = t.empty(max(n, 1), dtype=t.float64, device=self.device)
        dof = np.empty(coords.shape[0], dtype=np.int64)
        h = ctypes.c_void_p()
        st = self.lib.nn_assemble(self.handle, ctypes.byref(mesh), _ptr(D), nD, _ptr(ks), _ptr(f),
                                  _ptr(dmask), _ptr(dv), int(with_mass), ctypes.byref(h), _ptr(F),
                                  _ptr(dof))
        self._check(st, "nn_assemble")
        return self._wrap(h.value), F[:n], dof

    def matrix_from_csr(self, rowptr, col, val, mval=None) -> Matrix:
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        mval = None if mval is None else np.ascontiguousarray(mval, dtype=np.float64)
        h = ctypes.c_void_p()
        st = self.lib.nn_matrix_from_csr(self.handle, rowptr.size - 1, _ptr(rowptr), _ptr(col),
                                         _ptr(val), _ptr(mval), ctypes.byref(h))
        self._check(st, "nn_matrix_from_csr")
        return self._wrap(h.value)

    def _wrap(self, handle: int) -> Matrix:
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        hm = ctypes.c_int()
        self.lib.nn_matrix_info(handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(hm))
        return Matrix(self, handle, n.value, nnz.value, bool(hm.value))

    def matrix_export(self, A: Matrix):
        rowptr = np.empty(A.n + 1, dtype=np.int64)
        col = np.empty(max(A.nnz, 1), dtype=np.int32)
        val = np.empty(max(A.nnz, 1), dtype=np.float64)
        mval = np.empty(max(A.nnz, 1), dtype=np.float64) if A.has_mass else None
        st = self.lib.nn_matrix_export(self.handle, A.handle, _ptr(rowptr), _ptr(col), _ptr(val),
                                       _ptr(mval))
        self._check(st, "nn_matrix_export")
        m = A.nnz
        return rowptr, col[:m], val[:m], (None if mval is None else mval[:m])

    def matrix_bytes(self, A: Matrix, precision: int = NN_FP64) -> int:
        b = ctypes.c_size_t()
        self._check(self.lib.nn_matrix_bytes(A.handle, precision, ctypes.byref(b)), "nn_matrix_bytes")
        return int(b.value)

    # ---------------------------------------------------------------- compute
    def matvec(self, A: Matrix, x, which: int = 0, out=None):
        t = self.torch
        y = out if out is not None else t.empty(max(A.n, 1), dtype=t.float64, device=self.device)
        self._check(self.lib.nn_matvec(self.handle, A.handle, which, _ptr(x), _ptr(y)), "nn_matvec")
        return y[:A.n]

    def solve_nonneg(self, A: Matrix, f, opts: Optional[Opts] = None, c=None, active=None,
                     allow_maxit: bool = False, **kw):
        """Returns (c, active, stats dict).  `c` (device float64) is used as the
        warm start when opts.c0_mode == 1 and overwritten with the solution."""
        t = self.torch
        o = opts if opts is not None else default_opts(**kw)
        if c is None:
            c = t.zeros(max(A.n, 1), dtype=t.float64, device=self.device)
        if active is None:
            active = t.empty(max(A.n, 1), dtype=t.uint8, device=self.device)
        st_out = Stats()
        st = self.lib.nn_solve_nonneg(self.handle, A.handle, _ptr(f), ctypes.byref(o), _ptr(c),
                                      _ptr(active), ctypes.byref(st_out))
        self._check(st, "nn_solve_nonneg", allow=(NN_OK, NN_EMAXIT) if allow_maxit else (NN_OK,))
        d = st_out.as_dict()
        d["status"] = st
        return c[:A.n], active[:A.n], d

    def solve_nonneg_noalloc(self, A: Matrix, f, c, active, opts: Optional[Opts] = None,
                             allow_maxit: bool = False, **kw):
        """nn_solve_nonneg_noalloc: the same solve with the library's fixed
        work array (no device allocation inside the call; n <= 262,144).
        The caller passes c (warm start when opts.c0_mode == 1, overwritten
        with the solution) and active.  Returns (c, active, stats dict)."""
        o = opts if opts is not None else default_opts(**kw)
        st_out = Stats()
        st = self.lib.nn_solve_nonneg_noalloc(self.handle, A.handle, _ptr(f), ctypes.byref(o),
                                              _ptr(c), _ptr(active), ctypes.byref(st_out))
        self._check(st, "nn_solve_nonneg_noalloc",
                    allow=(NN_OK, NN_EMAXIT) if allow_maxit else (NN_OK,))
        d = st_out.as_dict()
        d["status"] = st
        return c[:A.n], active[:A.n], d

    def solve_galerkin(self, A: Matrix, f, opts: Optional[Opts] = None, c=None,
                       allow_maxit: bool = False, **kw):
        """Unconstrained Galerkin solve K c = f (nn_solve_galerkin).  Returns
        (c, stats dict); stats carry min_c, max_c, n_negative and the true
        relative residual in kkt_rel."""
        t = self.torch
        o = opts if opts is not None else default_opts(**kw)
        if c is None:
            c = t.empty(max(A.n, 1), dtype=t.float64, device=self.device)
        st_out = Stats()
        st = self.lib.nn_solve_galerkin(self.handle, A.handle, _ptr(f), ctypes.byref(o), _ptr(c),
                                        ctypes.byref(st_out))
        self._check(st, "nn_solve_galerkin", allow=(NN_OK, NN_EMAXIT) if allow_maxit else (NN_OK,))
        d = st_out.as_dict()
        d["status"] = st
        return c[:A.n], d

    def step_transient(self, A: Matrix, dt: float, f, c, opts: Optional[Opts] = None,
                       active=None, allow_maxit: bool = False, **kw):
        t = self.torch
        o = opts if opts is not None else default_opts(**kw)
        if active is None:
            active = t.empty(max(A.n, 1), dtype=t.uint8, device=self.device)
        st_out = Stats()
        st = self.lib.nn_step_transient(self.handle, A.handle, float(dt), _ptr(f), ctypes.byref(o),
                                        _ptr(c), _ptr(active), ctypes.byref(st_out))
        self._check(st, "nn_step_transient", allow=(NN_OK, NN_EMAXIT) if allow_maxit else (NN_OK,))
        d = st_out.as_dict()
        d["status"] = st
        return c[:A.n], active[:A.n], d

    def solve_batch(self, As, fs, opts: Optional[Opts] = None, cs=None, actives=None,
                    allow_fail: bool = False, **kw):
        """Solve len(As) independent problems with one batched call
        (nn_solve_batch).  Returns (cs, actives, stats list, status).  Each
        c in `cs` (device float64, one per problem) is the warm start when
        opts.c0_mode == 1 and is overwritten with that member's solution."""
        t = self.torch
        o = opts if opts is not None else default_opts(**kw)
        P = len(As)
        if len(fs) != P:
            raise ValueError("one load vector per matrix")
        if cs is None:
            cs = [t.zeros(max(A.n, 1), dtype=t.float64, device=self.device) for A in As]
        if actives is None:
            actives = [t.empty(max(A.n, 1), dtype=t.uint8, device=self.device) for A in As]
        arr = ctypes.c_void_p * max(P, 1)
        Ka = arr(*[A.handle for A in As])
        fa = arr(*[_ptr(f) for f in fs])
        ca = arr(*[_ptr(c) for c in cs])
        aa = arr(*[_ptr(a) for a in actives])
        st_arr = (Stats * max(P, 1))()
        st = self.lib.nn_solve_batch(self.handle, P, Ka, fa, ctypes.byref(o), ca, aa, st_arr)
        if not allow_fail:
            self._check(st, "nn_solve_batch")
        stats = [st_arr[k].as_dict() for k in range(P)]
        return ([c[:A.n] for c, A in zip(cs, As)], [a[:A.n] for a, A in zip(actives, As)],
                stats, st)

    def step_transient_batch(self, As, dt: float, fs, cs, opts: Optional[Opts] = None,
                             actives=None, allow_fail: bool = False, **kw):
        """One backward-Euler step of every member (nn_step_transient_batch):
        each c in `cs` holds c^n and is overwritten with c^(n+1).  Returns
        (cs, actives, stats list, status)."""
        t = self.torch
        o = opts if opts is not None else default_opts(**kw)
        P = len(As)
        if len(fs) != P or len(cs) != P:
            raise ValueError("one load and one state vector per matrix")
        if actives is None:
            actives = [t.empty(max(A.n, 1), dtype=t.uint8, device=self.device) for A in As]
        arr = ctypes.c_void_p * max(P, 1)
        st_arr = (Stats * max(P, 1))()
        st = self.lib.nn_step_transient_batch(
            self.handle, P, arr(*[A.handle for A in As]), float(dt), arr(*[_ptr(f) for f in fs]),
            ctypes.byref(o), arr(*[_ptr(c) for c in cs]), arr(*[_ptr(a) for a in actives]), st_arr)
        if not allow_fail:
            self._check(st, "nn_step_transient_batch")
        return ([c[:A.n] for c, A in zip(cs, As)], [a[:A.n] for a, A in zip(actives, As)],
                [st_arr[k].as_dict() for k in range(P)], st)

    # ---------------------------------------------------------------- profiling
    def set_profiling(self, on, classes=None, every: int = 1):
        """Time kernel launches with HIP events: on=False stops; `classes`
        (names from KCLASS_NAMES) limits timing to those classes; `every`
        times one launch in `every` of the CG classes (nn_set_profiling_sample)."""
        mask = 0
        if on:
            mask = NN_PROF_ALL if classes is None else sum(1 << KCLASS_NAMES.index(c) for c in classes)
        self._check(self.lib.nn_set_profiling_sample(self.handle, int(every)), "nn_set_profiling_sample")
        self._check(self.lib.nn_set_profiling(self.handle, mask), "nn_set_profiling")

    def kernel_times(self, reset: bool = False) -> dict:
        counts = np.zeros(NN_KCLASSES, dtype=np.int64)
        ms = np.zeros(NN_KCLASSES)
        by = np.zeros(NN_KCLASSES)
        bc = np.zeros(NN_KCLASSES)
        self._check(self.lib.nn_kernel_times(self.handle, _ptr(counts), _ptr(ms), _ptr(by),
                                             _ptr(bc), int(reset)), "nn_kernel_times")
        return {name: {"count": int(counts[k]), "ms": float(ms[k]), "bytes": float(by[k]),
                       "bytes_csr": float(bc[k])}
                for k, name in enumerate(KCLASS_NAMES)}
