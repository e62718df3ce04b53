"""Batched solves: many systems of uneven sizes with several right-hand sides in one
context, against single-system solves and dense solutions."""
import numpy as np
import pytest

from paper_1904_04093_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_04093_amd import gabp
    gabp.load()
    return gabp


def _family(nsys, lo, hi, nrhs, seed):
    fam = W.batch_family(nsys=nsys, nrhs=nrhs, side_lo=lo, side_hi=hi, seed=seed)
    systems = [a for a, _ in fam]
    rhs = [bb for _, bb in fam]
    return systems, rhs


def _stack(rhs, nrhs):
    return torch.as_tensor(np.stack([np.concatenate([r[q] for r in rhs]) for q in range(nrhs)])).cuda()


@pytest.mark.parametrize("mode,nrhs", [("joint", 1), ("joint", 4), ("precomp", 2), ("precomp", 4)])
def test_batch_matches_single_solves(B, mode, nrhs):
    systems, rhs = _family(7, 8, 21, nrhs, seed=31)
    kw = dict(mode=mode, check_every=8)
    if mode == "precomp":
        kw.update(tol_lambda=0.0, max_lambda_sweeps=60)
    bs = B.BatchSolver(systems, nrhs=nrhs, **kw)
    X, infos = bs.solve(_stack(rhs, nrhs), 1e-11, 50000)
    X = X.cpu().numpy()
    off = bs.offsets
    for s, a in enumerate(systems):
        single = B.Solver.from_csr(a, **kw)
        for q in range(nrhs):
            xs, info = single.solve(torch.as_tensor(rhs[s][q]).cuda(), 1e-11, 50000)
            xb = X[q, off[s]:off[s + 1]]
            xs = xs.cpu().numpy()
            assert infos[s * nrhs + q].status == B.OK
            assert infos[s * nrhs + q].sweeps == info.sweeps, (s, q)
            assert np.abs(xb - xs).max() <= 1e-12 * np.abs(xs).max(), (s, q)


@pytest.mark.parametrize("nrhs", [1, 4])
def test_batch_ir_reaches_dense_solutions(B, nrhs):
    systems, rhs = _family(9, 8, 40, nrhs, seed=32)
    bs = B.BatchSolver(systems, nrhs=nrhs, mode="precomp", precision="f32_ir", check_every=16,
                       tol_lambda=1e-8)
    X, infos = bs.solve(_stack(rhs, nrhs), 1e-10, 400000)
    X = X.cpu().numpy()
    off = bs.offsets
    for s, a in enumerate(systems):
        A = W.csr_to_dense(a)
        for q in range(nrhs):
            info = infos[s * nrhs + q]
            assert info.status == B.OK and info.rel_res2 <= 1e-10, (s, q, info)
            xs = np.linalg.solve(A, rhs[s][q])
            assert np.abs(X[q, off[s]:off[s + 1]] - xs).max() <= 1e-7 * np.abs(xs).max()
    # systems of different sizes finish after different sweep counts
    sweeps = sorted(i.sweeps for i in infos)
    assert sweeps[0] < sweeps[-1]


def test_batch_rejects_coupled_systems(B):
    a, _ = W.small_upwind(8)
    lib = B.load()
    import ctypes
    off = np.array([0, 30, 64], dtype=np.int32)      # a row of system 0 couples to system 1
    h = ctypes.c_void_p()
    o = B._options()
    st = lib.gabp_setup_batched(ctypes.byref(h), 2, off.ctypes.data_as(ctypes.c_void_p), a.n,
                                a.nnz, a.rowptr.ctypes.data_as(ctypes.c_void_p),
                                a.col.ctypes.data_as(ctypes.c_void_p),
                                a.val.ctypes.data_as(ctypes.c_void_p), 1, ctypes.byref(o), None)
    assert st == B.EINVAL


@pytest.fixture(scope="module")
def full_family():
    return _family(512, 48, 384, 4, seed=3)


@pytest.mark.parametrize("mode", ["joint", "precomp"])
def test_batch_full_shape_sampled_parity(B, full_family, mode):
    """The full batching shape (512 systems, sides 48..384, 28.2M unknowns, 4 right-hand
    sides) in one context, with the kernel variants the batched benchmark runs at that size
    (non-temporal streams, 2-byte reverse deltas): after 5 sweeps (FP64, joint or with 30
    precomputed Lt sweeps) the smallest, the largest and one random system match the oracle
    for every right-hand side."""
    from oracle import gabp as G
    systems, rhs = full_family
    k, klam = 5, 30
    kw = dict(mode=mode, check_every=k)
    if mode == "precomp":
        kw.update(precision="f64", tol_lambda=0.0, max_lambda_sweeps=klam)
    bs = B.BatchSolver(systems, nrhs=4, **kw)
    X, infos = bs.solve(_stack(rhs, 4), 1e-30, k)
    X = X.cpu().numpy()
    off = bs.offsets
    sizes = np.array([a.n for a in systems])
    picks = {int(np.argmin(sizes)), int(np.argmax(sizes)),
             int(W.rng(330, 0).integers(0, len(systems)))}
    for s in sorted(picks):
        g = G.Graph.from_csr(systems[s])
        lam = G.lambda_phase(g, 0.0, klam)[:2] if mode == "precomp" else None
        for q in range(4):
            assert infos[s * 4 + q].sweeps == k, (s, q, infos[s * 4 + q])
            b = rhs[s][q]
            if lam is None:
                xo, _, _ = G.run(g, b, k)
            else:
                m = np.zeros(g.E)
                for _ in range(k):
                    xo, m = G.msweep(g, b, lam[0], lam[1], m)
            xb = X[q, off[s]:off[s + 1]]
            assert np.abs(xb - xo).max() <= 1e-12 * np.abs(xo).max(), (mode, s, q)
