"""Thin ctypes binding of libamge.so (include/amge.h); argument marshalling only.

Every numerical step of the solve phase runs in the library's HIP kernels; this
module converts Python arguments to the C ABI.  Device vectors are torch CUDA
(HIP) tensors passed by pointer; streams are torch streams; by default the library's
device memory comes from torch's caching allocator (amge_opts.alloc).  There is no
Python or CPU fallback: if the library is missing, importing the binding raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np
# torch is loaded before the library: torch ships its own HIP runtime, and the library's
# runtime dependency then resolves to that one (a process that loads the library first
# holds two HIP runtimes, and device allocations through the library's can fail).
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamge.so")

CURL, DIV = 0, 1
OK, NOT_CONVERGED, CANCELLED = 0, 1, 2   # request statuses that are not errors
OP_A, OP_AHAT, OP_D, OP_DT, OP_P, OP_PT, OP_SMOOTH, OP_SMOOTHT, OP_COARSE, OP_SWEEP, OP_RESID = range(11)

STATUS = {0: "AMGE_OK", 1: "AMGE_NOT_CONVERGED", 2: "AMGE_CANCELLED", -1: "AMGE_ERR_ARG", -2: "AMGE_ERR_SHAPE",
          -3: "AMGE_ERR_NOT_SPD", -4: "AMGE_ERR_OOM", -5: "AMGE_ERR_HIP", -6: "AMGE_ERR_BREAKDOWN",
          -7: "AMGE_ERR_NONFINITE", -8: "AMGE_ERR_BUSY"}


class AmgeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class CsrC(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class LevelC(C.Structure):
    _fields_ = [("A", CsrC), ("D", CsrC), ("P", CsrC)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEALLOC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class OptsC(C.Structure):
    _fields_ = [("nu_primary", C.c_int32), ("nu_aux", C.c_int32), ("precond_bits", C.c_int32),
                ("max_rhs", C.c_int32), ("tail_rows", C.c_int32), ("smoother", C.c_int32),
                ("resid_bits", C.c_int32), ("alloc", ALLOC_FN), ("dealloc", DEALLOC_FN), ("alloc_user", C.c_void_p)]


SMOOTHERS = {"l1jacobi": 0, "symgs": 1, "l1blockgs": 2}


def _torch_alloc(nbytes, _user):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes))
    except Exception:   # out of memory: the library reports AMGE_ERR_OOM
        return None


def _torch_dealloc(ptr, _user):
    torch.cuda.caching_allocator_delete(ptr)


# torch's caching allocator as the library's device allocator (kept alive for the process)
TORCH_ALLOC = (ALLOC_FN(_torch_alloc), DEALLOC_FN(_torch_dealloc))


class CompletionC(C.Structure):
    _fields_ = [("tag", C.c_int64), ("hierarchy", C.c_int32), ("status", C.c_int32), ("iters", C.c_int32),
                ("pad", C.c_int32), ("relres", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2107_05613_amd.build")
    lib = C.CDLL(LIB_PATH)
    vp, i32, f64 = C.c_void_p, C.c_int32, C.c_double
    sig = {
        "amge_default_opts": (None, [C.POINTER(OptsC)]),
        "amge_setup_hierarchy": (i32, [C.POINTER(LevelC), i32, C.POINTER(OptsC), vp, C.POINTER(vp)]),
        "amge_destroy": (None, [vp]),
        "amge_ctx_create": (i32, [vp, i32, C.POINTER(vp)]),
        "amge_ctx_destroy": (None, [vp]),
        "amge_footprint": (i32, [vp, i32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "amge_vcycle": (i32, [vp, vp, vp, i32, vp]),
        "amge_vcycle_static": (i32, [vp, vp, vp, vp]),
        "amge_pcg_solve": (i32, [vp, vp, vp, i32, f64, i32, i32, C.POINTER(i32), C.POINTER(f64), vp]),
        "amge_level_apply": (i32, [vp, i32, i32, i32, vp, vp, vp, vp]),
        "amge_hierarchy_info": (i32, [vp, C.POINTER(i32), C.POINTER(i32)]),
        "amge_precision_info": (i32, [vp, C.POINTER(f64), C.POINTER(i32), C.POINTER(i32)]),
        "amge_timing_enable": (i32, [vp, i32]),
        "amge_vcycle_bytes": (i32, [vp, i32, i32, C.POINTER(f64)]),
        "amge_timing_read": (i32, [vp, C.POINTER(f64), C.POINTER(C.c_int64), C.POINTER(f64)]),
        "amge_last_error": (C.c_char_p, []),
        "amge_kuhn_build": (i32, [i32, i32, i32, C.POINTER(f64), C.POINTER(f64), i32, C.POINTER(vp)]),
        "amge_problem_nlevels": (i32, [vp]),
        "amge_problem_levels": (i32, [vp, C.POINTER(LevelC)]),
        "amge_problem_free": (None, [vp]),
        "amge_server_create": (i32, [C.c_size_t, C.c_size_t, i32, C.POINTER(vp)]),
        "amge_server_destroy": (None, [vp]),
        "amge_server_add": (i32, [vp, vp, C.POINTER(i32)]),
        "amge_server_add_grouped": (i32, [vp, vp, i32, C.POINTER(i32)]),
        "amge_server_ensemble": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "amge_server_request_bytes": (i32, [vp, i32, C.POINTER(C.c_size_t)]),
        "amge_server_submit": (i32, [vp, i32, vp, vp, f64, i32, i32, C.c_int64, vp]),
        "amge_server_progress": (i32, [vp, i32, C.POINTER(CompletionC), i32, C.POINTER(i32)]),
        "amge_server_stats": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_size_t),
                                    C.POINTER(C.c_size_t)]),
        "amge_server_cancel": (i32, [vp, C.c_int64, C.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()

# Objects still open at interpreter exit are closed before torch shuts down (their device
# memory goes back through torch's allocator): servers first, then contexts, then
# hierarchies.  Registered after torch's own exit handlers, so it runs before them.
_LIVE = {"server": weakref.WeakSet(), "context": weakref.WeakSet(), "hierarchy": weakref.WeakSet()}


@atexit.register
def _close_all():
    for kind in ("server", "context", "hierarchy"):
        for obj in list(_LIVE[kind]):
            try:
                obj.close()
            except Exception:
                pass

# Names declared by include/amge.h (checked by the test suite against the header).
EXPORTS = ("amge_default_opts", "amge_setup_hierarchy", "amge_destroy", "amge_ctx_create", "amge_ctx_destroy",
           "amge_footprint", "amge_vcycle", "amge_vcycle_static",
           "amge_pcg_solve", "amge_level_apply", "amge_hierarchy_info", "amge_precision_info", "amge_last_error",
           "amge_timing_enable", "amge_timing_read", "amge_vcycle_bytes",
           "amge_kuhn_build", "amge_problem_nlevels", "amge_problem_levels", "amge_problem_free",
           "amge_server_create", "amge_server_destroy", "amge_server_add", "amge_server_add_grouped",
           "amge_server_ensemble", "amge_server_request_bytes", "amge_server_submit", "amge_server_progress",
           "amge_server_stats", "amge_server_cancel")


def lib():
    return _lib


def _check(code, allow=(0,)):
    if code in allow:
        return code
    raise AmgeError(code, _lib.amge_last_error().decode())


def _ptr(t):
    """Device pointer of a torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _vec(t, n):
    """Device pointer of a contiguous FP64 CUDA tensor holding at least n entries."""
    if isinstance(t, int):
        return t
    if t.dtype.itemsize != 8 or not t.is_floating_point() or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if t.numel() < n:
        raise ValueError(f"tensor holds {t.numel()} entries, need {n}")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------------------------------- problems
class HostCsr:
    """Host CSR arrays (numpy), FP64 values, int32 indices."""

    def __init__(self, nrows, ncols, rowptr, col, val):
        self.shape = (int(nrows), int(ncols))
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)

    @property
    def nnz(self):
        return len(self.col)

    @classmethod
    def from_scipy(cls, M):
        M = M.tocsr()
        M.sort_indices()
        return cls(M.shape[0], M.shape[1], M.indptr, M.indices, M.data)

    def to_c(self):
        c = CsrC()
        c.nrows, c.ncols, c.nnz = self.shape[0], self.shape[1], self.nnz
        c.rowptr = self.rowptr.ctypes.data_as(C.POINTER(C.c_int32))
        c.col = self.col.ctypes.data_as(C.POINTER(C.c_int32))
        c.val = self.val.ctypes.data_as(C.POINTER(C.c_double))
        return c

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=self.shape)


def _csr_copy(c: CsrC):
    nr, nnz = c.nrows, c.nnz
    rp = np.ctypeslib.as_array(c.rowptr, (nr + 1,)).copy() if nr else np.zeros(1, np.int32)
    ci = np.ctypeslib.as_array(c.col, (nnz,)).copy() if nnz else np.zeros(0, np.int32)
    va = np.ctypeslib.as_array(c.val, (nnz,)).copy() if nnz else np.zeros(0)
    return HostCsr(nr, c.ncols, rp, ci, va)


BUILD_ESSENTIAL, BUILD_COEFFICIENT, BUILD_DEVICE = 1, 2, 4


def build_problem(kind, n, nlevels, alpha_hex, beta_hex, extension="l2", bc="natural", device=False):
    """Structured workload (amge_kuhn_build): per level (A, D, P) as HostCsr, P None on the last.
    extension: "l2" or "coefficient" (weighted local problems); bc: "natural" or "essential";
    device: the set-up work of AMGE_BUILD_DEVICE on the current GPU."""
    k = {"curl": CURL, "div": DIV}.get(kind, kind)
    if extension not in ("l2", "coefficient") or bc not in ("natural", "essential"):
        raise ValueError("extension must be 'l2' or 'coefficient', bc 'natural' or 'essential'")
    flags = ((BUILD_COEFFICIENT if extension == "coefficient" else 0) | (BUILD_ESSENTIAL if bc == "essential" else 0)
             | (BUILD_DEVICE if device else 0))
    a = np.ascontiguousarray(alpha_hex, dtype=np.float64)
    b = np.ascontiguousarray(beta_hex, dtype=np.float64)
    if a.size != n ** 3 or b.size != n ** 3:
        raise ValueError("alpha_hex and beta_hex need n**3 values")
    h = C.c_void_p()
    _check(_lib.amge_kuhn_build(k, n, nlevels, a.ctypes.data_as(C.POINTER(C.c_double)),
                                b.ctypes.data_as(C.POINTER(C.c_double)), flags, C.byref(h)))
    try:
        L = _lib.amge_problem_nlevels(h)
        arr = (LevelC * L)()
        _check(_lib.amge_problem_levels(h, arr))
        out = []
        for i, lv in enumerate(arr):
            P = _csr_copy(lv.P) if i + 1 < L else None
            out.append((_csr_copy(lv.A), _csr_copy(lv.D), P))
        return out
    finally:
        _lib.amge_problem_free(h)


# ----------------------------------------------------------------------------- hierarchy
class Hierarchy:
    """Device-resident AMGe hierarchy (amge_setup_hierarchy): the read-only level
    operators.  Solves run on contexts (Context, amge_ctx_create); the hierarchy's own
    methods vcycle / pcg / level_apply / timing_* use a default context of max_rhs
    columns, created on first use.

    precond_bits: 32, 64 or 0 (chosen by trial solves at set-up); max_rhs: widest block
    of a context (the batched path); tail_rows: levels of at most this many rows below the
    fine one are folded into one dense FP64 operator (0: every level runs its kernels);
    smoother: "l1jacobi", "symgs" (symmetric Gauss-Seidel in colour order) or "l1blockgs"
    (l1-scaled symmetric block Gauss-Seidel, 64-row blocks); "symgs" runs single-column
    contexts only; resid_bits: precision of an FP32 V-cycle's fine-level residual (32,
    64, or 0: 32 unless the trial picks 64); allocator: "torch" (torch's caching
    allocator) or None (hipMalloc)."""

    def __init__(self, levels, nu_primary=2, nu_aux=2, precond_bits=32, max_rhs=1, tail_rows=2048, stream=None,
                 allocator="torch", smoother="l1jacobi", resid_bits=0):
        L = len(levels)
        arr = (LevelC * L)()
        self._keep = []
        for i, (A, D, P) in enumerate(levels):
            mats = []
            for M in (A, D, P):
                if M is None:
                    M = HostCsr(0, 0, np.zeros(1, np.int32), [], [])
                elif not isinstance(M, HostCsr):
                    M = HostCsr.from_scipy(M)
                mats.append(M)
            self._keep.extend(mats)
            arr[i].A, arr[i].D, arr[i].P = (m.to_c() for m in mats)
        if allocator == "torch":
            al, de = TORCH_ALLOC
        elif allocator is None:
            al, de = ALLOC_FN(), DEALLOC_FN()
        else:
            raise ValueError("allocator must be 'torch' or None")
        opts = OptsC(nu_primary, nu_aux, precond_bits, max_rhs, tail_rows, SMOOTHERS[smoother], resid_bits, al, de,
                     None)
        h = C.c_void_p()
        _check(_lib.amge_setup_hierarchy(arr, L, C.byref(opts), _stream(stream), C.byref(h)))
        self._h = h
        self._keep = None
        self._ctx = None
        self.opts = opts
        self.max_rhs = max_rhs
        nl = C.c_int32()
        rows = (C.c_int32 * L)()
        _check(_lib.amge_hierarchy_info(h, C.byref(nl), rows))
        self.rows = list(rows)
        self.nlevels = nl.value
        _LIVE["hierarchy"].add(self)

    def close(self):
        if getattr(self, "_ctx", None) is not None:
            self._ctx.close()
            self._ctx = None
        if getattr(self, "_h", None):
            _lib.amge_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def context(self, nrhs=1):
        """A new context (work buffers, stream, captured graphs) for up to nrhs columns."""
        return Context(self, nrhs)

    @property
    def ctx(self):
        """The default context (max_rhs columns)."""
        if self._ctx is None:
            self._ctx = Context(self, self.max_rhs)
        return self._ctx

    def precision_info(self):
        """(kappa, precond_bits in use)."""
        k, b = C.c_double(), C.c_int32()
        _check(_lib.amge_precision_info(self._h, C.byref(k), C.byref(b), None))
        return k.value, b.value

    def resid_bits(self):
        """Precision of an FP32 V-cycle's fine-level residual (32 or 64; 64 for FP64 V-cycles)."""
        r = C.c_int32()
        _check(_lib.amge_precision_info(self._h, None, None, C.byref(r)))
        return r.value

    def footprint_parts(self, nrhs=None):
        """(hierarchy bytes, bytes of one context of nrhs columns; default max_rhs)."""
        hb, cb = C.c_size_t(), C.c_size_t()
        _check(_lib.amge_footprint(self._h, int(nrhs or self.max_rhs), C.byref(hb), C.byref(cb)))
        return hb.value, cb.value

    def footprint(self, nrhs=None):
        """Device bytes of the hierarchy and one context of nrhs columns (default max_rhs)."""
        return sum(self.footprint_parts(nrhs))

    def vcycle_bytes(self, precision=32, nrhs=1):
        v = C.c_double()
        _check(_lib.amge_vcycle_bytes(self._h, precision, nrhs, C.byref(v)))
        return v.value

    def vcycle(self, r, z, nrhs=1, stream=None):
        self.ctx.vcycle(r, z, nrhs=nrhs, stream=stream)

    def vcycle_static(self, r, z, stream=None):
        """z = B r on one column with the library's static scratch (amge_vcycle_static):
        no context, no device allocation."""
        n = self.rows[0]
        _check(_lib.amge_vcycle_static(self._h, _vec(r, n), _vec(z, n), _stream(stream)))

    def pcg(self, b, x, rtol=1e-8, maxit=500, stop_norm=0, nrhs=1, stream=None):
        return self.ctx.pcg(b, x, rtol=rtol, maxit=maxit, stop_norm=stop_norm, nrhs=nrhs, stream=stream)

    def level_apply(self, level, op, x, out, x2=None, precision=64, stream=None):
        self.ctx.level_apply(level, op, x, out, x2=x2, precision=precision, stream=stream)

    def timing_enable(self, on=True):
        self.ctx.timing_enable(on)

    def timing_read(self):
        return self.ctx.timing_read()


class Context:
    """Execution context of a hierarchy (amge_ctx_create): the solve calls run here.
    Contexts of one hierarchy may run concurrently (different streams or threads)."""

    def __init__(self, H: Hierarchy, nrhs=1):
        c = C.c_void_p()
        _check(_lib.amge_ctx_create(H.handle, int(nrhs), C.byref(c)))
        self._c = c
        self.H = H            # the hierarchy outlives its contexts
        self.nrhs = nrhs
        self.rows = H.rows
        _LIVE["context"].add(self)

    def close(self):
        if getattr(self, "_c", None):
            _lib.amge_ctx_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._c

    def vcycle(self, r, z, nrhs=1, stream=None):
        """z = B r (one V-cycle) on n_1 x nrhs row-major FP64 device blocks."""
        n = self.rows[0] * nrhs
        _check(_lib.amge_vcycle(self._c, _vec(r, n), _vec(z, n), nrhs, _stream(stream)))

    def pcg(self, b, x, rtol=1e-8, maxit=500, stop_norm=0, nrhs=1, stream=None):
        """Returns (status, iters[nrhs], relres[nrhs]); status 0 or 1 (not converged)."""
        it = (C.c_int32 * nrhs)()
        rr = (C.c_double * nrhs)()
        n = self.rows[0] * nrhs
        code = _check(_lib.amge_pcg_solve(self._c, _vec(b, n), _vec(x, n), nrhs, float(rtol), int(maxit),
                                          int(stop_norm), it, rr, _stream(stream)), allow=(0, 1))
        return code, list(it), list(rr)

    def timing_enable(self, on=True):
        _check(_lib.amge_timing_enable(self._c, 1 if on else 0))

    def timing_read(self):
        """(ms, launches, algorithmic bytes) of the fine-level A kernels since the last read."""
        ms, n, by = C.c_double(), C.c_int64(), C.c_double()
        _check(_lib.amge_timing_read(self._c, C.byref(ms), C.byref(n), C.byref(by)))
        return ms.value, n.value, by.value

    def level_apply(self, level, op, x, out, x2=None, precision=64, stream=None):
        _check(_lib.amge_level_apply(self._c, level, op, precision, _ptr(x), _ptr(x2), _ptr(out),
                                     _stream(stream)))


# ----------------------------------------------------------------------------- serving
class Server:
    """Serving engine (amge_server_*): resident hierarchies, continuous batching of
    single right-hand-side requests.  Hierarchies passed to add() must have max_rhs >= 2
    and must outlive the server; they are used only by it."""

    def __init__(self, hierarchy_budget=0, inflight_budget=0, chunk=8):
        h = C.c_void_p()
        _check(_lib.amge_server_create(int(hierarchy_budget), int(inflight_budget), int(chunk), C.byref(h)))
        self._h = h
        self._rows = []
        self._hier = []
        self._cap = 256
        self._buf = (CompletionC * self._cap)()
        _LIVE["server"].add(self)

    def close(self):
        if getattr(self, "_h", None):
            _lib.amge_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, H: "Hierarchy", grouped=False, ensemble=0) -> int:
        """grouped: H joins ensemble number `ensemble`, whose members' iterations share
        grouped launches."""
        i = C.c_int32()
        if grouped:
            _check(_lib.amge_server_add_grouped(self._h, H.handle, int(ensemble), C.byref(i)))
        else:
            _check(_lib.amge_server_add(self._h, H.handle, C.byref(i)))
        self._rows.append(H.rows[0])
        self._hier.append(H)
        return i.value

    def request_bytes(self, hid) -> int:
        b = C.c_size_t()
        _check(_lib.amge_server_request_bytes(self._h, hid, C.byref(b)))
        return b.value

    def submit(self, hid, b, x, tag, rtol=1e-8, maxit=500, stop_norm=0, stream=None):
        n = self._rows[hid]
        _check(_lib.amge_server_submit(self._h, hid, _vec(b, n), _vec(x, n), float(rtol), int(maxit),
                                       int(stop_norm), int(tag), _stream(stream)))

    def progress(self, wait=True):
        """Completed requests as a list of (tag, hierarchy, status, iters, relres)."""
        out = []
        while True:
            k = C.c_int32()
            _check(_lib.amge_server_progress(self._h, 1 if (wait and not out) else 0, self._buf, self._cap,
                                             C.byref(k)))
            for c in self._buf[:k.value]:
                out.append((c.tag, c.hierarchy, c.status, c.iters, c.relres))
            if k.value < self._cap:
                return out

    def ensemble(self):
        """Summed over the ensembles: (members, kernels per grouped iteration, kernels of
        the members' own iterations)."""
        m, k, k1 = C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.amge_server_ensemble(self._h, C.byref(m), C.byref(k), C.byref(k1)))
        return m.value, k.value, k1.value

    def cancel(self, tag) -> int:
        """Cancels the unfinished requests with this tag (amge_server_cancel); returns how
        many.  Each still completes, once, with status CANCELLED."""
        n = C.c_int32()
        _check(_lib.amge_server_cancel(self._h, int(tag), C.byref(n)))
        return n.value

    def stats(self):
        q, f = C.c_int32(), C.c_int32()
        fb, rb = C.c_size_t(), C.c_size_t()
        _check(_lib.amge_server_stats(self._h, C.byref(q), C.byref(f), C.byref(fb), C.byref(rb)))
        return {"queued": q.value, "inflight": f.value, "inflight_bytes": fb.value, "resident_bytes": rb.value}
