"""Python binding of libgabp (ctypes). Argument marshalling only.

Every step of the solver runs in the HIP library; PyTorch supplies device memory (CUDA
tensors on ROCm) and the current stream. If the library is missing the import of this
module succeeds but every call raises: there is no CPU fallback.

Entry points mirror ``include/gabp.h``; see that header for the meaning of each argument.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgabp.so")

OK, MAXSWEEPS = 0, 1
EINVAL, ENOMEM, EZERODIAG, ENUMERIC, EDEVICE, ENOTSUPP = -1, -2, -3, -4, -5, -6
MODES = {"joint": 0, "precomp": 1, "seq": 2}
PRECISIONS = {"f64": 0, "f32_ir": 1}
SCHEDULES = {"flood": 0, "redblack": 1, "lines": 2, "lines_alt": 3}


class GaBPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gabp status {status}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("tol_lambda", ctypes.c_double),
                ("max_lambda_sweeps", ctypes.c_int32),
                ("ir_inner_tol", ctypes.c_double), ("ir_max_inner", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("grid_nx", ctypes.c_int32), ("grid_ny", ctypes.c_int32),
                ("tiles", ctypes.c_int32), ("block", ctypes.c_int32),
                ("progress_s", ctypes.c_double), ("stream_hints", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("lambda_sweeps", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("rel_res2", ctypes.c_double), ("res_inf", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PI64 = ctypes.POINTER(ctypes.c_int64)

_SIGS = {
    "gabp_default_options": (None, [ctypes.POINTER(Options)]),
    "gabp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "gabp_last_error": (ctypes.c_char_p, []),
    "gabp_validate_csr": (ctypes.c_int, [_I32, _I64, _P, _P, _P, _P]),
    "gabp_setup": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _I64, _P, _P, _P, _P, _P,
                                  ctypes.POINTER(Options), _P]),
    "gabp_update_values": (ctypes.c_int, [_P, _P, _P]),
    "gabp_destroy": (None, [_P]),
    "gabp_solve": (ctypes.c_int, [_P, _P, _P, _D, _I32, ctypes.POINTER(Info), _P]),
    "gabp_solve_transposed": (ctypes.c_int, [_P, _P, _P, _D, _I32, ctypes.POINTER(Info), _P]),
    "gabp_sweeps": (ctypes.c_int, [_P, _P, _P, _I32, _I32, _I32, _P]),
    "gabp_precompute_lambda": (ctypes.c_int, [_P, _I32, _PI32, _P]),
    "gabp_smooth": (ctypes.c_int, [_P, _P, _P, _I32, _P]),
    "gabp_residual": (ctypes.c_int, [_P, _P, _P, _P, _I32, _P, _P]),
    "gabp_residual_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _I32, _P, _P]),
    "gabp_adjoint_scatter": (ctypes.c_int, [_P, _P, _P, _P, _I32, _P, _P, _P, _P, _P]),
    "gabp_get_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_size_t), _P]),
    "gabp_set_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "gabp_residual_history": (ctypes.c_int, [_P, _P, _I32, _PI32]),
    "gabp_get_messages": (ctypes.c_int, [_P, _P, _P, _P]),
    "gabp_layout_info": (ctypes.c_int, [_P, _PI32, _PI64, _PI64, _PI64, _PI32]),
    "gabp_copy_probe": (ctypes.c_int, [_P, _P, _I64, _P]),
    "gabp_autotune": (ctypes.c_int, [_P, _PI32, _PI32, _PI32, _P]),
    "gabp_setup_batched": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _P, _I32, _I64, _P, _P, _P,
                                          _I32, ctypes.POINTER(Options), _P]),
    "gabp_solve_batched": (ctypes.c_int, [_P, _P, _P, _D, _I32, _P, _P]),
    "mg_setup": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _P, _P, _I32, _I32, _I32, _P]),
    "mg_vcycle": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(_D), _P]),
    "mg_solve": (ctypes.c_int, [_P, _P, _P, _D, _I32, _PI32, ctypes.POINTER(_D), _P]),
    "mg_destroy": (None, [_P]),
}

_lib = None


def load():
    """Load libgabp.so (torch first, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libgabp.so is not built ({LIB_PATH}); run "
                           "`python -m paper_1904_04093_amd.build`")
    try:
        import torch  # noqa: F401  (loads the HIP runtime torch was built with)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols():
    return list(_SIGS)


def _check(status, allow=(OK,)):
    if status in allow:
        return status
    msg = load().gabp_last_error().decode() or load().gabp_strerror(status).decode()
    raise GaBPError(status, msg)


def _host(a, dtype):
    arr = np.ascontiguousarray(np.asarray(a), dtype=dtype)
    return arr, arr.ctypes.data_as(_P)


def validate_csr(n, rowptr, col, val, rev=None) -> int:
    """Host-side CSR check (no GPU). Returns the status code."""
    rp, prp = _host(rowptr, np.int32)
    c, pc = _host(col, np.int32)
    v, pv = _host(val, np.float64)
    if rev is not None:
        r, pr = _host(rev, np.int32)
    else:
        r, pr = None, None
    return load().gabp_validate_csr(int(n), int(rp[-1]), prp, pc, pv, pr)


def _stream():
    import torch
    return _P(torch.cuda.current_stream().cuda_stream)


def _dev(t, n, dtype_name="float64"):
    import torch
    dt = getattr(torch, dtype_name)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dt or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"expected a contiguous {dtype_name} tensor with {n} elements")
    return _P(t.data_ptr())


def _check_jacobian(jptr, jnnz, jw, nnz):
    """The parameter Jacobian's index arrays must stay inside the matrix, since the library
    reads them on the device unchecked: jptr runs from 0 to len(jnnz) without decreasing,
    jw has one weight per jnnz entry and every jnnz lies in [0, nnz). Works on host or
    device tensors (a device check reads four scalars back)."""
    m = int(jnnz.numel())
    if int(jw.numel()) != m or int(jptr.numel()) < 1:
        raise ValueError("the parameter Jacobian needs len(jw) == len(jnnz) and a jptr")
    if int(jptr[0]) != 0 or int(jptr[-1]) != m or \
            (jptr.numel() > 1 and bool((jptr[1:] < jptr[:-1]).any())):
        raise ValueError("jptr must run from 0 to len(jnnz) without decreasing")
    if m and (int(jnnz.min()) < 0 or int(jnnz.max()) >= nnz):
        raise ValueError("jnnz must index stored entries: 0 <= jnnz < nnz")


def copy_probe(src, dst):
    """dst <- src with the library's plain streaming copy kernel (CUDA tensors, same size)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb or not (src.is_cuda and dst.is_cuda):
        raise ValueError("copy_probe needs two CUDA tensors of the same byte size")
    _check(load().gabp_copy_probe(_P(src.data_ptr()), _P(dst.data_ptr()), nb, _stream()))


@dataclass
class SolveInfo:
    status: int
    sweeps: int
    lambda_sweeps: int
    outer_iters: int
    rel_res2: float
    res_inf: float


class Solver:
    """One GaBP context on the current device for a CSR matrix (host arrays)."""

    def __init__(self, n, rowptr, col, val, rev=None, colour=None, *, mode="joint",
                 precision="f64", check_every=16, tol_lambda=1e-14,
                 max_lambda_sweeps=100000, ir_inner_tol=1e-4,
                 ir_max_inner=1000000, schedule="flood", use_graphs=True, grid=None,
                 progress_s=0.0, block=256, tiles=False, stream_hints=-1):
        lib = load()
        self._lib = lib
        o = Options()
        lib.gabp_default_options(ctypes.byref(o))
        o.mode, o.precision = MODES[mode], PRECISIONS[precision]
        o.check_every, o.tol_lambda = int(check_every), float(tol_lambda)
        o.max_lambda_sweeps = int(max_lambda_sweeps)
        o.ir_inner_tol, o.ir_max_inner = float(ir_inner_tol), int(ir_max_inner)
        o.schedule = SCHEDULES[schedule]
        o.use_graphs = int(bool(use_graphs))
        o.progress_s = float(progress_s)
        o.block = int(block)
        o.tiles = int(bool(tiles))
        o.stream_hints = int(stream_hints)
        if grid is not None:                  # (nx, ny) of the line schedules
            o.grid_nx, o.grid_ny = int(grid[0]), int(grid[1])
        self.options = o
        rp, prp = _host(rowptr, np.int32)
        c, pc = _host(col, np.int32)
        v, pv = _host(val, np.float64)
        self.n, self.nnz = int(n), int(rp[-1])
        pr = _host(rev, np.int32) if rev is not None else (None, None)
        pk = _host(colour, np.uint8) if colour is not None else (None, None)
        h = _P()
        _check(lib.gabp_setup(ctypes.byref(h), self.n, self.nnz, prp, pc, pv, pr[1], pk[1],
                              ctypes.byref(o), _stream()))
        self._h = h

    @classmethod
    def from_csr(cls, a, **kw):
        return cls(a.n, a.rowptr, a.col, a.val, **kw)

    # ---- lifecycle
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.gabp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, dtype="float64"):
        import torch
        return torch.empty(self.n, dtype=getattr(torch, dtype), device="cuda")

    # ---- solves
    def solve(self, b, tol, max_sweeps, x=None, transposed=False):
        x = self._new() if x is None else x
        info = Info()
        fn = self._lib.gabp_solve_transposed if transposed else self._lib.gabp_solve
        st = fn(self._h, _dev(b, self.n), _dev(x, self.n), float(tol), int(max_sweeps),
                ctypes.byref(info), _stream())
        _check(st, allow=(OK, MAXSWEEPS))
        return x, SolveInfo(**info.as_dict())

    def solve_transposed(self, g, tol, max_sweeps, lam=None):
        return self.solve(g, tol, max_sweeps, x=lam, transposed=True)

    def sweeps(self, b, sweeps, reset=True, transposed=False, x=None):
        x = self._new() if x is None else x
        _check(self._lib.gabp_sweeps(self._h, _dev(b, self.n), _dev(x, self.n), int(sweeps),
                                     int(bool(reset)), int(bool(transposed)), _stream()))
        return x

    def precompute_lambda(self, transposed=False):
        k = ctypes.c_int32(0)
        _check(self._lib.gabp_precompute_lambda(self._h, int(bool(transposed)),
                                                ctypes.byref(k), _stream()))
        return k.value

    def smooth(self, b, x, mu):
        _check(self._lib.gabp_smooth(self._h, _dev(b, self.n), _dev(x, self.n), int(mu),
                                     _stream()))
        return x

    def residual(self, b, x, transposed=False, want_r=True, want_norms=True):
        """r = b - A x (or b - A^T x) and, with want_norms, (||r||_2, ||r||_inf, ||b||_2)
        read back to the host (which waits for the stream); without, only enqueued."""
        r = self._new() if want_r else None
        norms = (ctypes.c_double * 3)() if want_norms else None
        _check(self._lib.gabp_residual(self._h, _dev(b, self.n), _dev(x, self.n),
                                       _dev(r, self.n) if want_r else None,
                                       int(bool(transposed)), norms, _stream()))
        return r, tuple(norms) if want_norms else None

    def residual_noalloc(self, b, x, r=None, norms=None, transposed=False):
        """gabp_residual_noalloc: r = b - A x and the norms into caller-owned device tensors
        (r: n doubles, norms: 3 doubles; either may be None); nothing is read back."""
        _check(self._lib.gabp_residual_noalloc(
            self._h, _dev(b, self.n), _dev(x, self.n),
            _dev(r, self.n) if r is not None else None, int(bool(transposed)),
            _dev(norms, 3) if norms is not None else None, _stream()))
        return r, norms

    def adjoint_scatter(self, lam, x, jac=None, want_G=True):
        import torch
        G = torch.empty(self.nnz, dtype=torch.float64, device="cuda") if want_G else None
        dtheta = None
        args = [None, 0, None, None, None, None]
        if jac is not None:
            jptr, jnnz, jw = jac
            _check_jacobian(jptr, jnnz, jw, self.nnz)
            npar = int(jptr.numel()) - 1
            dtheta = torch.empty(npar, dtype=torch.float64, device="cuda")
            args = [_dev(jptr, npar + 1, "int32"), _dev(jnnz, jnnz.numel(), "int32"),
                    _dev(jw, jw.numel()), _dev(dtheta, npar)]
            _check(self._lib.gabp_adjoint_scatter(
                self._h, _dev(lam, self.n), _dev(x, self.n),
                _dev(G, self.nnz) if want_G else None, npar, *args, _stream()))
        else:
            _check(self._lib.gabp_adjoint_scatter(
                self._h, _dev(lam, self.n), _dev(x, self.n), _dev(G, self.nnz), 0,
                None, None, None, None, _stream()))
        return G, dtheta

    values_version = 0          # bumped by every update_values (autograd checks it)

    def update_values(self, val):
        _check(self._lib.gabp_update_values(self._h, _dev(val, self.nnz), _stream()))
        self.values_version += 1

    def get_state(self) -> bytes:
        nb = ctypes.c_size_t(0)
        _check(self._lib.gabp_get_state(self._h, None, ctypes.byref(nb), _stream()))
        buf = ctypes.create_string_buffer(nb.value)
        _check(self._lib.gabp_get_state(self._h, buf, ctypes.byref(nb), _stream()))
        return buf.raw[: nb.value]

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._lib.gabp_set_state(self._h, buf, len(blob), _stream()))

    def messages(self):
        """(Lt, m) of the current message state in setup CSR order (device tensors of nnz
        doubles; see gabp_get_messages)."""
        import torch
        lam = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        msg = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        _check(self._lib.gabp_get_messages(self._h, _dev(lam, self.nnz), _dev(msg, self.nnz),
                                           _stream()))
        return lam, msg

    def residual_history(self):
        """||r||_2 / ||b||_2 at every check of the last solve (numpy array)."""
        import numpy as np
        cnt = ctypes.c_int32(0)
        _check(self._lib.gabp_residual_history(self._h, None, 0, ctypes.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.float64)
        if cnt.value:
            _check(self._lib.gabp_residual_history(
                self._h, out.ctypes.data_as(_P), cnt.value, ctypes.byref(cnt)))
        return out

    def autotune(self):
        """Pick streaming hints, workgroup size and the check interval by measurement (see
        gabp_autotune)."""
        ce, hints, blk = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        _check(self._lib.gabp_autotune(self._h, ctypes.byref(ce), ctypes.byref(hints),
                                       ctypes.byref(blk), _stream()))
        return {"check_every": ce.value, "stream_hints": hints.value, "block": blk.value}

    def layout_info(self):
        n, nnz, slots, pad = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        rb = ctypes.c_int32()
        _check(self._lib.gabp_layout_info(self._h, ctypes.byref(n), ctypes.byref(nnz),
                                          ctypes.byref(slots), ctypes.byref(pad), ctypes.byref(rb)))
        return {"n": n.value, "nnz": nnz.value, "slots": slots.value, "padded_slots": pad.value,
                "rev_bytes": rb.value}

    @property
    def handle(self):
        return self._h


def _options(mode="joint", precision="f64", check_every=16, tol_lambda=1e-14,
             max_lambda_sweeps=100000, ir_inner_tol=1e-4, ir_max_inner=1000000,
             schedule="flood", use_graphs=True):
    o = Options()
    load().gabp_default_options(ctypes.byref(o))
    o.mode, o.precision = MODES[mode], PRECISIONS[precision]
    o.check_every, o.tol_lambda = int(check_every), float(tol_lambda)
    o.max_lambda_sweeps = int(max_lambda_sweeps)
    o.ir_inner_tol, o.ir_max_inner = float(ir_inner_tol), int(ir_max_inner)
    o.schedule = SCHEDULES[schedule]
    o.use_graphs = int(bool(use_graphs))
    return o


class BatchSolver:
    """Independent systems (a list of CSR matrices) with nrhs right-hand sides each, solved
    together by one block-diagonal context."""

    def __init__(self, systems, nrhs=1, **opts):
        lib = load()
        self._lib = lib
        sizes = [int(a.n) for a in systems]
        off = np.zeros(len(systems) + 1, dtype=np.int64)
        off[1:] = np.cumsum(sizes)
        rps, cols, vals = [np.zeros(1, dtype=np.int64)], [], []
        base = 0
        for a, o in zip(systems, off[:-1]):
            rps.append(a.rowptr[1:].astype(np.int64) + base)
            cols.append(a.col.astype(np.int64) + o)
            vals.append(a.val)
            base += int(a.rowptr[-1])
        rowptr = np.concatenate(rps)
        col = np.concatenate(cols)
        val = np.concatenate(vals)
        if off[-1] >= 2**31 or rowptr[-1] >= 2**31:
            raise ValueError("batch too large for int32 indices")
        self.nsys, self.nrhs, self.n = len(systems), int(nrhs), int(off[-1])
        self.offsets = off
        o = _options(**opts)
        self.options = o
        so, pso = _host(off, np.int32)
        rp, prp = _host(rowptr, np.int32)
        c, pc = _host(col, np.int32)
        v, pv = _host(val, np.float64)
        h = _P()
        _check(lib.gabp_setup_batched(ctypes.byref(h), self.nsys, pso, self.n, int(rp[-1]),
                                      prp, pc, pv, self.nrhs, ctypes.byref(o), _stream()))
        self._h = h

    def autotune(self):
        ce, hints, blk = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        _check(self._lib.gabp_autotune(self._h, ctypes.byref(ce), ctypes.byref(hints),
                                       ctypes.byref(blk), _stream()))
        return {"check_every": ce.value, "stream_hints": hints.value, "block": blk.value}

    def solve(self, B, tol, max_sweeps, X=None):
        """B, X: CUDA float64 tensors of shape (nrhs, n). Returns X and per-pair infos."""
        import torch
        X = torch.empty(self.nrhs, self.n, dtype=torch.float64, device="cuda") if X is None else X
        infos = (Info * (self.nsys * self.nrhs))()
        st = self._lib.gabp_solve_batched(self._h, _dev(B, self.nrhs * self.n),
                                          _dev(X, self.nrhs * self.n), float(tol),
                                          int(max_sweeps), infos, _stream())
        _check(st, allow=(OK, MAXSWEEPS, ENUMERIC))
        out = [SolveInfo(**i.as_dict()) for i in infos]
        return X, out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.gabp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SMOOTHERS = {"gabp": 0, "rbgs": 1}


class Multigrid:
    """V-cycle over per-level Solver contexts (finest first) with a GaBP or RB-GS smoother."""

    def __init__(self, solvers, sides, smoother="gabp", nu1=2, nu2=2):
        lib = load()
        self._lib = lib
        self.solvers = list(solvers)          # keep the borrowed contexts alive
        self.sides = [int(s) for s in sides]
        arr = (_P * len(self.solvers))(*[s.handle for s in self.solvers])
        sd = (ctypes.c_int32 * len(self.sides))(*self.sides)
        h = _P()
        _check(lib.mg_setup(ctypes.byref(h), len(self.solvers), ctypes.cast(arr, _P),
                            ctypes.cast(sd, _P), SMOOTHERS[smoother], int(nu1), int(nu2),
                            _stream()))
        self._h = h
        self.n = self.solvers[0].n

    def vcycle(self, b, x):
        rel = ctypes.c_double(0.0)
        _check(self._lib.mg_vcycle(self._h, _dev(b, self.n), _dev(x, self.n),
                                   ctypes.byref(rel), _stream()))
        return rel.value

    def solve(self, b, tol, max_cycles, x=None):
        import torch
        x = torch.empty(self.n, dtype=torch.float64, device="cuda") if x is None else x
        cyc = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        st = self._lib.mg_solve(self._h, _dev(b, self.n), _dev(x, self.n), float(tol),
                                int(max_cycles), ctypes.byref(cyc), ctypes.byref(rel),
                                _stream())
        _check(st, allow=(OK, MAXSWEEPS, ENUMERIC))
        return x, {"status": st, "cycles": cyc.value, "rel_res2": rel.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
