"""Temporal blocking of the flood schedule (opt.tiles): two sweeps per launch over tiles of
13 grid rows x 64 columns (26 rows for FP32 messages), the first sweep's messages kept in LDS and the tile's halo rows
swept once more to supply them. The iterates must be those of plain flood sweeps: against
the FP64 oracle to 1e-12 (joint, frozen and per-sweep precomputed Lt, transposed), bit for
bit against the untiled layout, with every output slot written (poisoned buffers), and at
the benchmark's full size on sampled read-offs and messages."""
import json

import numpy as np
import pytest

from oracle import gabp as G
from paper_1904_04093_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_04093_amd import gabp
    gabp.load()
    return gabp


def _cuda(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64)).cuda()


def _rel_inf(x, y):
    return float(np.abs(np.asarray(x) - y).max() / max(np.abs(y).max(), 1e-300))


def _grids():
    out = {}
    a, b = W.small_upwind(32)
    out["upwind32"] = (a, b, 32, 32)                        # 1 x 3 tiles, x padding
    a, b = W.precision_at_scale(45)
    out["field45"] = (a, b, 45, 45)                         # ragged in x and y
    a = W.random_grid_5pt(130, 70, W.rng(330, 0), one_way=0.15, flip=0.2)
    out["rand130x70"] = (a, W.rng(330, 1).uniform(-1, 1, a.n), 130, 70)   # 3 x 6 tiles
    a = W.random_grid_5pt(200, 3, W.rng(330, 2))
    out["strip200x3"] = (a, W.rng(330, 3).uniform(-1, 1, a.n), 200, 3)    # one tile row
    return out


GRIDS = _grids()


@pytest.mark.parametrize("name", list(GRIDS))
def test_tiled_joint_sweeps_match_oracle(B, name):
    a, b, nx, ny = GRIDS[name]
    s = B.Solver.from_csr(a, tiles=True, grid=(nx, ny))
    g = G.Graph.from_csr(a)
    gt = g.transposed()
    bt = _cuda(b)
    for sweeps in (1, 2, 3, 10, 101):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        xo, Lt, m = G.run(g, b, sweeps)
        assert _rel_inf(x, xo) <= TOL, (name, sweeps)
        lam, msg = (t.cpu().numpy() for t in s.messages())
        idx = np.nonzero((a.row_of_nnz() != a.col) & (a.val != 0.0))[0]
        assert _rel_inf(lam[idx], Lt) <= TOL and _rel_inf(msg[idx], m) <= TOL, (name, sweeps)
        xt = s.sweeps(bt, sweeps, transposed=True).cpu().numpy()
        xot, _, _ = G.run(gt, b, sweeps)
        assert _rel_inf(xt, xot) <= TOL, (name, sweeps, "transposed")


@pytest.mark.parametrize("kw", [dict(mode="precomp", tol_lambda=0.0, max_lambda_sweeps=30),
                                dict(mode="seq")])
def test_tiled_mean_sweeps_match_oracle(B, kw):
    a, b, nx, ny = GRIDS["rand130x70"]
    s = B.Solver.from_csr(a, tiles=True, grid=(nx, ny), **kw)
    g = G.Graph.from_csr(a)
    bt = _cuda(b)
    for sweeps in (1, 2, 5, 12):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        if kw["mode"] == "seq":
            xo, _, _ = G.run(g, b, sweeps)
        else:
            Lt, S, _ = G.lambda_phase(g, 0.0, 30)
            m = np.zeros(g.E)
            for _ in range(sweeps):
                xo, m = G.msweep(g, b, Lt, S, m)
        assert _rel_inf(x, xo) <= TOL, (kw, sweeps)


@pytest.mark.parametrize("kw", [dict(mode="joint"),
                                dict(mode="precomp", tol_lambda=1e-12),
                                dict(mode="seq"),
                                dict(mode="precomp", precision="f32_ir", tol_lambda=1e-7)])
def test_tiled_equals_untiled_bitwise(B, monkeypatch, kw):
    """Same operations in the same order: sweeps (even and odd counts, continued without a
    reset), a solve's sweep count and iterate, and the same with every output buffer
    poisoned first (each slot a sweep reads was written by the sweep before)."""
    a, b, nx, ny = GRIDS["field45"]
    bt = _cuda(b)
    plain = B.Solver.from_csr(a, check_every=8, **kw)
    tiled = B.Solver.from_csr(a, check_every=8, tiles=True, grid=(nx, ny), **kw)
    monkeypatch.setenv("GABP_FAULT_INJECT", "poison-outputs")
    poisoned = B.Solver.from_csr(a, check_every=8, tiles=True, grid=(nx, ny), **kw)
    monkeypatch.delenv("GABP_FAULT_INJECT")
    for k, reset in ((2, True), (7, True), (5, False), (1, False)):
        want = plain.sweeps(bt, k, reset=reset).cpu().numpy()
        assert np.array_equal(tiled.sweeps(bt, k, reset=reset).cpu().numpy(), want), (k, kw)
        got = poisoned.sweeps(bt, k, reset=reset).cpu().numpy()
        assert np.all(np.isfinite(got)) and np.array_equal(got, want), (k, kw, "poisoned")
    if kw["mode"] != "seq":
        xw, iw = plain.solve(bt, 1e-9, 200000)
        for s in (tiled, poisoned):
            xg, ig = s.solve(bt, 1e-9, 200000)
            assert ig.status == iw.status and ig.sweeps == iw.sweeps
            assert np.array_equal(xg.cpu().numpy(), xw.cpu().numpy())


@pytest.mark.parametrize("kw", [dict(mode="joint"),
                                dict(mode="precomp", precision="f32_ir", tol_lambda=1e-7)])
def test_tiled_xcd_order_covers_every_tile(B, monkeypatch, kw):
    """A grid wide enough for several strips in the XCD-aware tile order, the last strip
    narrower (650 columns: 11 tile columns in strips of 2): every tile is taken exactly once
    (poisoned output buffers) and the iterates equal the untiled layout's bit for bit."""
    a = W.random_grid_5pt(650, 40, W.rng(333, 0))
    bt = _cuda(W.rng(333, 1).uniform(-1, 1, a.n))
    plain = B.Solver.from_csr(a, **kw)
    monkeypatch.setenv("GABP_FAULT_INJECT", "poison-outputs")
    tiled = B.Solver.from_csr(a, tiles=True, grid=(650, 40), **kw)
    monkeypatch.delenv("GABP_FAULT_INJECT")
    for k in (2, 3, 8):
        got = tiled.sweeps(bt, k).cpu().numpy()
        assert np.all(np.isfinite(got)) and np.array_equal(got, plain.sweeps(bt, k).cpu().numpy()), k


@pytest.mark.parametrize("kw", [dict(mode="joint"), dict(mode="seq"),
                                dict(mode="precomp", precision="f32_ir", tol_lambda=1e-7)])
def test_tiled_autotune(B, tmp_path, monkeypatch, kw):
    """The autotuner times a tiled layout with its two-sweep kernels under a cache entry of
    its own (the untiled layout of the same matrix gets another one), and the tuned kernels
    keep the iterates."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("GABP_AUTOTUNE_CACHE", str(cache))
    a, b, nx, ny = GRIDS["rand130x70"]
    bt = _cuda(b)
    ref = B.Solver.from_csr(a, **kw).sweeps(bt, 7).cpu().numpy()
    tiled = B.Solver.from_csr(a, tiles=True, grid=(nx, ny), **kw)
    plain = B.Solver.from_csr(a, **kw)
    t = tiled.autotune()
    plain.autotune()
    assert t["stream_hints"] in (0, 1, 2) and t["check_every"] in (8, 16, 32, 64, 128, 256)
    keys = [json.loads(line)["key"] for line in cache.read_text().splitlines()]
    assert len(keys) == 2 and keys[0] != keys[1]
    assert np.array_equal(tiled.sweeps(bt, 7).cpu().numpy(), ref)
    assert np.array_equal(plain.sweeps(bt, 7).cpu().numpy(), ref)


@pytest.mark.parametrize("kw", [dict(mode="joint"), dict(mode="seq"),
                                dict(mode="precomp", tol_lambda=1e-12),
                                dict(mode="seq", precision="f32_ir")])
def test_tiled_smoother_equals_untiled(B, kw):
    """Algorithm 3 on a tiled layout (two-sweep launches, a plain one for an odd count, the
    correction added by the last launch): the same bits as the untiled smoother, against
    the oracle's joint smoother to 1e-12 in FP64."""
    a, b, nx, ny = GRIDS["rand130x70"]
    g = G.Graph.from_csr(a)
    bt = _cuda(b)
    plain = B.Solver.from_csr(a, **kw)
    tiled = B.Solver.from_csr(a, tiles=True, grid=(nx, ny), **kw)
    x0 = W.rng(334, 0).uniform(-1, 1, a.n)
    xp, xt = _cuda(x0), _cuda(x0)
    xo = x0.copy()
    for mu in (1, 2, 3, 4):
        plain.smooth(bt, xp, mu)
        tiled.smooth(bt, xt, mu)
        assert np.array_equal(xt.cpu().numpy(), xp.cpu().numpy()), (kw, mu)
        if kw["mode"] in ("joint", "seq") and "precision" not in kw:
            xo = G.smooth(g, b, xo, mu)
            assert _rel_inf(xt.cpu().numpy(), xo) <= TOL, (kw, mu)


@pytest.mark.parametrize("kw", [dict(mode="joint"), dict(mode="precomp", tol_lambda=1e-12),
                                dict(mode="precomp", precision="f32_ir", tol_lambda=1e-7)])
def test_tiled_cache_hints_keep_the_bits(B, kw):
    """The three cache-hint settings of the tiled kernels (plain; non-temporal loads and
    stores; non-temporal stores only) compute the same bits; the third needs a tiled
    layout."""
    a, b, nx, ny = GRIDS["rand130x70"]
    bt = _cuda(b)
    outs = [B.Solver.from_csr(a, tiles=True, grid=(nx, ny), stream_hints=h, **kw)
            .sweeps(bt, 7).cpu().numpy() for h in (0, 1, 2)]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    with pytest.raises(B.GaBPError):
        B.Solver.from_csr(a, stream_hints=2, **kw)
    with pytest.raises(B.GaBPError):
        B.Solver.from_csr(a, tiles=True, grid=(nx, ny), stream_hints=3, **kw)


def test_tiled_options_are_checked(B):
    a, b, nx, ny = GRIDS["upwind32"]
    with pytest.raises(B.GaBPError):
        B.Solver.from_csr(a, tiles=True)                       # no grid
    with pytest.raises(B.GaBPError):
        B.Solver.from_csr(a, tiles=True, grid=(16, 32))       # grid does not match n
    with pytest.raises(B.GaBPError):
        B.Solver.from_csr(a, tiles=True, grid=(nx, ny), schedule="redblack",
                          colour=W.grid_colouring(32))
    a9 = W.random_grid_9pt(20, 20, W.rng(331, 0))
    with pytest.raises(B.GaBPError) as e:
        B.Solver.from_csr(a9, tiles=True, grid=(20, 20))     # 8 neighbours per row
    assert e.value.status == B.ENOTSUPP


def _ball_problem(a, b, j, radius):
    seen = {int(j)}
    frontier = [int(j)]
    for _ in range(radius):
        nxt = []
        for u in frontier:
            for c in a.col[a.rowptr[u]:a.rowptr[u + 1]]:
                c = int(c)
                if c not in seen:
                    seen.add(c)
                    nxt.append(c)
        frontier = nxt
    nodes = np.array(sorted(seen))
    rows = []
    for u in nodes:
        lo, hi = a.rowptr[u], a.rowptr[u + 1]
        keep = np.isin(a.col[lo:hi], nodes)
        rows.append((np.searchsorted(nodes, a.col[lo:hi][keep]), a.val[lo:hi][keep]))
    rp = np.zeros(len(nodes) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(c) for c, _ in rows])
    sub = W.CSR(len(nodes), rp, np.concatenate([c for c, _ in rows]).astype(np.int32),
                np.concatenate([v for _, v in rows]))
    return sub, b[nodes], int(np.searchsorted(nodes, j))


def test_tiled_full_size_sampled_parity(B):
    """The benchmark's 2048 x 2048 operator in its benchmark configuration (tiled, joint
    FP64): read-offs after 2, 3 and 16 sweeps at sampled nodes (tile corners, tile edges,
    grid corners, random) against the oracle on the radius-s ball around each."""
    n = 2048
    a, b = W.precision_at_scale(n)
    s = B.Solver.from_csr(a, tiles=True, grid=(n, n))
    bt = _cuda(b)
    r = W.rng(332, 0)
    pick = [0, n - 1, n * n - 1, n * (n - 1), 63, 64, 12 * n + 63, 13 * n + 64, 13 * n + 63,
            12 * n + 64, 25 * n + 127, 26 * n + 128, 2047 * n - 1000, 31 * n + 1000]
    samples = np.concatenate([np.array(pick), r.choice(n * n, 30, replace=False)])
    for sweeps in (2, 3, 16):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        for j in samples:
            sub, sb, sj = _ball_problem(a, b, j, sweeps)
            xo, _, _ = G.run(G.Graph.from_csr(sub), sb, sweeps)
            assert abs(x[j] - xo[sj]) <= TOL * max(abs(xo[sj]), 1e-300) + 1e-300, (j, sweeps)
