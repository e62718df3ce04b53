"""The C-ABI library loads, exports every symbol include/gabp.h declares, and its host-only
entry points behave (no GPU needed: nothing here launches a kernel)."""
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from paper_1904_04093_amd import gabp as B
from paper_1904_04093_amd import workloads as W

HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b((?:gabp|mg)_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    declared = _declared()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), f"{name} declared but not exported"
    assert set(declared) == set(B.declared_symbols()), "binding and header disagree"


def test_strerror_and_defaults():
    lib = B.load()
    assert lib.gabp_strerror(0) == b"ok"
    assert b"diagonal" in lib.gabp_strerror(-3)
    o = B.Options()
    lib.gabp_default_options(o)
    assert o.check_every == 16 and o.mode == 0 and o.tol_lambda == 1e-14
    # the last fields: the binding's struct has the header's layout
    assert o.tiles == 0 and o.block == 256 and o.progress_s == 0.0 and o.stream_hints == -1


def _rev(a):
    d = {}
    rows = a.row_of_nnz()
    for e, (i, j) in enumerate(zip(rows, a.col)):
        d[(int(i), int(j))] = e
    return np.array([d.get((int(j), int(i)), -1) for i, j in zip(rows, a.col)], dtype=np.int32)


def test_validate_csr_accepts_good_input():
    a, _ = W.small_upwind(8)
    assert B.validate_csr(a.n, a.rowptr, a.col, a.val) == B.OK
    assert B.validate_csr(a.n, a.rowptr, a.col, a.val, _rev(a)) == B.OK
    # structurally nonsymmetric matrix with its rev index (-1 where A_ji is absent)
    r = W.rng(200, 0)
    b = W.random_walk_summable(50, 0.1, r)
    assert B.validate_csr(b.n, b.rowptr, b.col, b.val, _rev(b)) == B.OK


def test_validate_csr_rejects_bad_input():
    a, _ = W.small_upwind(6)
    val = a.val.copy()
    diag = np.nonzero(a.row_of_nnz() == a.col)[0]
    val[diag[3]] = 0.0
    assert B.validate_csr(a.n, a.rowptr, a.col, val) == B.EZERODIAG
    # missing diagonal
    A = W.csr_to_dense(a)
    A[5, 5] = 0.0
    m = W.csr_from_dense(A)
    assert B.validate_csr(m.n, m.rowptr, m.col, m.val) == B.EZERODIAG
    # unsorted columns
    col = a.col.copy()
    col[[0, 1]] = col[[1, 0]]
    assert B.validate_csr(a.n, a.rowptr, col, a.val) == B.EINVAL
    # out of range column
    col = a.col.copy()
    col[3] = a.n
    assert B.validate_csr(a.n, a.rowptr, col, a.val) == B.EINVAL
    # inconsistent reverse index
    rv = _rev(a)
    off = np.nonzero(rv >= 0)[0]
    rv[off[5]] = rv[off[6]]
    assert B.validate_csr(a.n, a.rowptr, a.col, a.val, rv) == B.EINVAL
    # non-finite value
    val = a.val.copy()
    val[2] = np.nan
    assert B.validate_csr(a.n, a.rowptr, a.col, val) == B.EINVAL
    # bad rowptr
    rp = a.rowptr.copy()
    rp[-1] += 1
    assert B.validate_csr(a.n, rp, np.append(a.col, 0), np.append(a.val, 1.0)) == B.EINVAL


def test_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        B._dev(torch.zeros(4, dtype=torch.float64), 4)


def _setup_status(a, opts, colour=None):
    """gabp_setup on host CSR arrays with the given options; the rejections below all
    happen in host code, before the library makes any HIP call."""
    import ctypes
    lib = B.load()
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(a.rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(a.col, dtype=np.int32)
    vl = np.ascontiguousarray(a.val, dtype=np.float64)
    ck = None if colour is None else np.ascontiguousarray(colour, dtype=np.uint8)
    st = lib.gabp_setup(ctypes.byref(h), a.n, a.nnz, rp.ctypes.data, cl.ctypes.data,
                        vl.ctypes.data, None, None if ck is None else ck.ctypes.data,
                        ctypes.byref(opts), None)
    assert not h.value, "a rejected set-up leaves no context"
    return st, lib.gabp_last_error().decode()


def _opts(**kw):
    o = B.Options()
    B.load().gabp_default_options(o)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@pytest.mark.parametrize("field,value", [
    ("check_every", 0), ("mode", 3), ("precision", 2), ("schedule", 9), ("block", 96),
    ("tiles", 2), ("stream_hints", 3), ("stream_hints", -2), ("ir_inner_tol", 0.0),
    ("ir_max_inner", 0), ("tol_lambda", -1.0), ("progress_s", float("nan"))])
def test_setup_rejects_invalid_options(field, value):
    a, _ = W.small_upwind(8)
    st, msg = _setup_status(a, _opts(**{field: value}))
    assert st == B.EINVAL and "invalid options" in msg


def test_setup_rejects_inconsistent_layout_requests():
    a, _ = W.small_upwind(8)
    # non-temporal stores only: a setting of the tiled kernels
    st, msg = _setup_status(a, _opts(stream_hints=2))
    assert st == B.EINVAL and "tiled" in msg
    # tiles: flood schedule, grid sides that multiply to n
    st, msg = _setup_status(a, _opts(tiles=1, grid_nx=8, grid_ny=8, schedule=B.SCHEDULES["redblack"]),
                            colour=(np.arange(64) + np.arange(64) // 8) % 2)
    assert st == B.EINVAL and "flood" in msg
    st, msg = _setup_status(a, _opts(tiles=1, grid_nx=8, grid_ny=7))
    assert st == B.EINVAL and "grid_nx" in msg
    st, msg = _setup_status(a, _opts(tiles=1))
    assert st == B.EINVAL and "grid_nx" in msg
    # rows wider than a tile's register budget (9-point stencil: 8 neighbours)
    g9 = W.random_grid_9pt(9, 9, W.rng(201, 0))
    st, msg = _setup_status(g9, _opts(tiles=1, grid_nx=9, grid_ny=9))
    assert st == B.ENOTSUPP and "neighbours" in msg
    # red-black without colours; per-sweep precision messages with a line schedule
    st, msg = _setup_status(a, _opts(schedule=B.SCHEDULES["redblack"]))
    assert st == B.EINVAL and "colours" in msg
    st, msg = _setup_status(a, _opts(mode=B.MODES["seq"], schedule=B.SCHEDULES["lines"],
                                     grid_nx=8, grid_ny=8))
    assert st == B.ENOTSUPP and "point schedules" in msg
    # colours at or above the supported number of classes
    st, msg = _setup_status(a, _opts(schedule=B.SCHEDULES["redblack"]), colour=np.full(64, 200))
    assert st == B.EINVAL and "colour" in msg


def _batched_status(a, sys_off, nrhs=1, opts=None):
    import ctypes
    lib = B.load()
    h = ctypes.c_void_p()
    so = np.ascontiguousarray(sys_off, dtype=np.int32)
    rp = np.ascontiguousarray(a.rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(a.col, dtype=np.int32)
    vl = np.ascontiguousarray(a.val, dtype=np.float64)
    st = lib.gabp_setup_batched(ctypes.byref(h), len(so) - 1, so.ctypes.data, a.n, a.nnz,
                                rp.ctypes.data, cl.ctypes.data, vl.ctypes.data, nrhs,
                                ctypes.byref(opts or _opts()), None)
    assert not h.value
    return st, lib.gabp_last_error().decode()


def test_batched_setup_rejects_bad_batches():
    """Host-side rejections of gabp_setup_batched (before any HIP call)."""
    a, _ = W.small_upwind(8)
    n = a.n
    assert _batched_status(a, [0, n], nrhs=3)[0] == B.EINVAL
    st, msg = _batched_status(a, [0, n], opts=_opts(schedule=B.SCHEDULES["lines"]))
    assert st == B.ENOTSUPP and "point schedules" in msg
    st, msg = _batched_status(a, [0, n], opts=_opts(mode=B.MODES["seq"]))
    assert st == B.ENOTSUPP
    st, msg = _batched_status(a, [0, n - 1])
    assert st == B.EINVAL and "0 to n" in msg
    st, msg = _batched_status(a, [0, 32, 32, n])
    assert st == B.EINVAL and "empty" in msg
    # the 8 x 8 grid split after row 30: row 30 couples to row 31 in the other system
    st, msg = _batched_status(a, [0, 31, n])
    assert st == B.EINVAL and "couples two systems" in msg
    # a bad CSR is caught before the system scan reads it
    col = a.col.copy()
    col[4] = n + 7
    bad = W.CSR(a.n, a.rowptr, col, a.val)
    assert _batched_status(bad, [0, n])[0] == B.EINVAL


def test_multigrid_setup_rejects_bad_hierarchies():
    """Host-side rejections of mg_setup that need no level context."""
    import ctypes
    lib = B.load()
    h = ctypes.c_void_p()
    ctxs = (ctypes.c_void_p * 3)()
    sides = np.array([15, 7, 3], dtype=np.int32)
    def status(levels, smoother=0, nu1=2, nu2=2):
        st = lib.mg_setup(ctypes.byref(h), levels, ctxs, sides.ctypes.data, smoother, nu1,
                          nu2, None)
        assert not h.value
        return st, lib.gabp_last_error().decode()
    st, msg = status(1)
    assert st == B.EINVAL and "two levels" in msg
    assert status(3, smoother=2)[0] == B.EINVAL
    assert status(3, nu1=-1)[0] == B.EINVAL
    st, msg = status(3)
    assert st == B.EINVAL and "NULL level context" in msg


def test_parameter_jacobian_is_checked_before_the_device_reads_it():
    """The binding rejects Jacobian index arrays that would make the parameter reduction
    read outside the stored entries (the library reads them on the device unchecked)."""
    torch = pytest.importorskip("torch")
    n = 8
    a, jptr, jnnz, jw = W.theta_jacobian(n, W.theta_problem(n, 0))
    jp, jn, w = torch.as_tensor(jptr), torch.as_tensor(jnnz), torch.as_tensor(jw)
    B._check_jacobian(jp, jn, w, a.nnz)              # the generator's Jacobian passes
    bad = jn.clone()
    bad[3] = a.nnz
    with pytest.raises(ValueError, match="jnnz"):
        B._check_jacobian(jp, bad, w, a.nnz)
    bad[3] = -1
    with pytest.raises(ValueError, match="jnnz"):
        B._check_jacobian(jp, bad, w, a.nnz)
    dec = jp.clone()
    dec[2], dec[3] = jp[3], jp[2] - 1
    with pytest.raises(ValueError, match="jptr"):
        B._check_jacobian(dec, jn, w, a.nnz)
    with pytest.raises(ValueError, match="jptr"):
        B._check_jacobian(jp[:-1], jn, w, a.nnz)
    with pytest.raises(ValueError, match="len"):
        B._check_jacobian(jp, jn, w[:-1], a.nnz)
