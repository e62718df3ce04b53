"""Pins of the two-layer (region) GaBP oracle, Sec. 3 / Algorithm 2 of arXiv 1904.04093
(no GPU).

References used: the ordinary GaBP oracle (itself pinned elsewhere) for the Bethe regions,
where the paper states the two-layer rules reduce to GaBP; exactness on trees of regions
(a single line, decoupled lines); the fixed-point theorem of Sec. 3.4 against numpy dense
solves; invariances derived from the update rules.
"""
import numpy as np
import pytest

from oracle import gabp as G
from oracle import regions as RG
from paper_1904_04093_amd import workloads as W


def _relerr(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / max(np.linalg.norm(y), 1e-300))


def _lines(a, nx, ny):
    return RG.RegionGraph(a, RG.grid_lines(nx, ny))


# --------------------------------------------------------------------------------------
# Bethe regions: the two-layer rules are ordinary GaBP (end of Sec. 3.2)
# --------------------------------------------------------------------------------------

def _bethe_vs_gabp(a_csr, b, sweeps):
    A = W.csr_to_dense(a_csr)
    rg = RG.RegionGraph(A, RG.edge_regions(A))
    g = G.Graph.from_csr(a_csr)
    edge = {(int(d), int(s)): e for e, (d, s) in enumerate(zip(g.dst, g.src))}
    lam, m = rg.zeros(), rg.zeros()
    Lt, mm = np.zeros(g.E), np.zeros(g.E)
    worst = 0.0
    for s in range(sweeps):
        x_r = RG.readoff(rg, b, lam, m)           # belief of the single-node regions
        _, _, lam, m = RG.sweep(rg, b, lam, m)
        x_g, Lt, mm, _, _ = G.sweep(g, b, Lt, mm)
        worst = max(worst, _relerr(x_r, x_g))
        for k, (i, j) in enumerate(rg.regions):
            for pos, (dst, src) in enumerate(((i, j), (j, i))):
                e = edge.get((int(dst), int(src)))
                want_l = Lt[e] * g.a_ji[e] if e is not None else 0.0
                want_m = mm[e] if e is not None else 0.0
                scale = 1.0 + abs(want_l) + abs(want_m)
                worst = max(worst, abs(lam[k][pos] - want_l) / scale,
                            abs(m[k][pos] - want_m) / scale)
    return worst


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bethe_regions_reduce_to_gabp(seed):
    r = W.rng(400, seed)
    a = W.random_walk_summable(14, 0.25, r)            # loopy, structurally nonsymmetric
    b = r.uniform(-1, 1, a.n)
    assert _bethe_vs_gabp(a, b, 7) < 1e-13


def test_bethe_regions_reduce_to_gabp_on_a_grid():
    a = W.random_grid_5pt(5, 4, W.rng(401, 0), one_way=0.2, flip=0.1)
    b = W.rng(401, 1).uniform(-1, 1, a.n)
    assert _bethe_vs_gabp(a, b, 6) < 1e-13


# --------------------------------------------------------------------------------------
# exactness when the region graph is a tree
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("grouped", [False, True])
@pytest.mark.parametrize("shape", [(17, 1), (1, 13)])
def test_single_line_is_solved_exactly(shape, grouped):
    # the read-off is the node's column solution: a single column is solved by the first
    # sweep; a single row needs the row's messages first (flood: the second sweep; rows
    # then columns: the first)
    nx, ny = shape
    a = W.random_grid_5pt(nx, ny, W.rng(402, nx), one_way=0.1, flip=0.2)
    b = W.rng(402, 7).uniform(-1, 1, a.n)
    rg = _lines(a, nx, ny)
    A = W.csr_to_dense(a)
    grp = RG.line_groups(nx, ny) if grouped else None
    x1, _, _ = RG.run(rg, b, 1, groups=grp)
    if ny == 1 and not grouped:
        assert np.allclose(x1, b / np.diag(A), rtol=1e-15, atol=0)    # zero messages: Jacobi
        x2, _, _ = RG.run(rg, b, 2, groups=grp)
        assert _relerr(x2, np.linalg.solve(A, b)) < 1e-13
    else:
        assert _relerr(x1, np.linalg.solve(A, b)) < 1e-13


@pytest.mark.parametrize("decouple", ["vertical", "horizontal"])
def test_decoupled_lines_are_exact_after_one_update(decouple):
    nx, ny = 9, 7
    kw = dict(ky=0.0) if decouple == "vertical" else dict(kx=0.0)
    a = W.random_grid_5pt(nx, ny, W.rng(403, 0), flip=0.2, **kw)
    b = W.rng(403, 1).uniform(-1, 1, a.n)
    rg = _lines(a, nx, ny)
    want = np.linalg.solve(W.csr_to_dense(a), b)
    x2, _, _ = RG.run(rg, b, 2)
    assert _relerr(x2, want) < 1e-13
    x1, _, _ = RG.run(rg, b, 1, groups=RG.line_groups(nx, ny))   # rows, then columns
    assert _relerr(x1, want) < 1e-13


def test_coupled_grid_is_not_exact_after_one_update():
    nx, ny = 9, 7
    a = W.random_grid_5pt(nx, ny, W.rng(404, 0))
    b = W.rng(404, 1).uniform(-1, 1, a.n)
    x2, _, _ = RG.run(_lines(a, nx, ny), b, 2)
    assert _relerr(x2, np.linalg.solve(W.csr_to_dense(a), b)) > 1e-3


# --------------------------------------------------------------------------------------
# fixed point = A^{-1} b (Sec. 3.4, consistency theorem), for every read-off
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["laplacian", "random_nonsym", "upwind"])
def test_fixed_point_is_the_solution(case):
    if case == "laplacian":
        nx = ny = 8
        a = W.laplacian_5pt(8)
    elif case == "random_nonsym":
        nx, ny = 10, 7
        a = W.random_grid_5pt(nx, ny, W.rng(405, 0), one_way=0.15, flip=0.1)
    else:
        nx = ny = 12
        a, _ = W.small_upwind(12)
    b = W.rng(405, 1).uniform(-1, 1, a.n)
    rg = _lines(a, nx, ny)
    want = np.linalg.solve(W.csr_to_dense(a), b)
    x, st, sweeps, rel = RG.solve(rg, b, 1e-13, 5000)
    assert st == RG.OK
    assert _relerr(x, want) < 1e-11
    _, xr, _, _ = RG.sweep(rg, b, *RG.run(rg, b, sweeps)[1:])
    for r, xl in zip(rg.regions, xr):
        assert np.allclose(xl, want[r], rtol=0, atol=1e-10 * np.abs(want).max())


def test_line_iteration_beats_point_gabp_on_an_anisotropic_grid():
    # strong horizontal coupling: the lines carry it exactly (Sec. 5 motivation)
    nx, ny = 48, 6
    a = W.random_grid_5pt(nx, ny, W.rng(406, 0), margin=0.02, kx=1.0, ky=0.01)
    b = W.rng(406, 1).uniform(-1, 1, a.n)
    _, st_l, sw_l, _ = RG.solve(_lines(a, nx, ny), b, 1e-10, 4000)
    _, info, _, _ = G.solve(G.Graph.from_csr(a), b, 1e-10, 4000)
    assert st_l == RG.OK and info.status == G.OK
    assert sw_l * 3 < info.sweeps


# --------------------------------------------------------------------------------------
# rows-then-columns schedule: one of the two interleaved chains of the flood schedule
# --------------------------------------------------------------------------------------

def test_rows_then_columns_is_one_chain_of_the_flood():
    # rows only touch columns, so flood row messages at step 2s-1 and column messages at
    # step 2s come from one chain; the grouped schedule runs exactly that chain
    nx, ny = 9, 7
    a = W.random_grid_5pt(nx, ny, W.rng(413, 0), one_way=0.15, flip=0.2)
    b = W.rng(413, 1).uniform(-1, 1, a.n)
    rg = _lines(a, nx, ny)
    grp = RG.line_groups(nx, ny)
    lf, mf = rg.zeros(), rg.zeros()
    flood = []
    for t in range(8):
        _, _, lf, mf = RG.sweep(rg, b, lf, mf)
        flood.append((lf, mf))
    la, ma = rg.zeros(), rg.zeros()
    for s in range(1, 5):
        _, _, la, ma = RG.sweep(rg, b, la, ma, groups=grp)
        fr_l, fr_m = flood[2 * s - 2]
        fc_l, fc_m = flood[2 * s - 1]
        for k in grp[0]:
            assert np.allclose(la[k], fr_l[k], rtol=1e-14, atol=1e-15)
            assert np.allclose(ma[k], fr_m[k], rtol=1e-14, atol=1e-15)
        for k in grp[1]:
            assert np.allclose(la[k], fc_l[k], rtol=1e-14, atol=1e-15)
            assert np.allclose(ma[k], fc_m[k], rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("precomp", [False, True])
def test_rows_then_columns_fixed_point(precomp):
    nx, ny = 10, 9
    a = W.random_grid_5pt(nx, ny, W.rng(414, 0), one_way=0.1, flip=0.1)
    b = W.rng(414, 1).uniform(-1, 1, a.n)
    rg = _lines(a, nx, ny)
    grp = RG.line_groups(nx, ny)
    pc = None
    if precomp:
        lam, invs, _ = RG.lambda_phase(rg, 1e-14, 2000, groups=grp)
        pc = (lam, invs)
    x, st, _, _ = RG.solve(rg, b, 1e-13, 5000, precomp=pc, groups=grp)
    assert st == RG.OK
    assert _relerr(x, np.linalg.solve(W.csr_to_dense(a), b)) < 1e-11


# --------------------------------------------------------------------------------------
# invariances of the update rules
# --------------------------------------------------------------------------------------

def test_row_scaling_sign_and_linearity():
    nx, ny = 7, 6
    a = W.random_grid_5pt(nx, ny, W.rng(407, 0), one_way=0.1, flip=0.2)
    r = W.rng(407, 1)
    b1, b2 = r.uniform(-1, 1, a.n), r.uniform(-1, 1, a.n)
    A = W.csr_to_dense(a)
    d = r.uniform(0.5, 2.0, a.n) * np.where(r.random(a.n) < 0.5, -1, 1)
    rg = _lines(a, nx, ny)
    for s in (1, 2, 3, 6):
        x1, _, _ = RG.run(rg, b1, s)
        xs, _, _ = RG.run(_lines(W.csr_from_dense(d[:, None] * A), nx, ny), d * b1, s)
        assert _relerr(xs, x1) < 1e-13                     # row scaling: same iterates
        xn, _, _ = RG.run(_lines(W.csr_from_dense(-A), nx, ny), -b1, s)
        assert _relerr(xn, x1) < 1e-14                     # (A, b) -> (-A, -b)
        x2, _, _ = RG.run(rg, b2, s)
        x12, _, _ = RG.run(rg, b1 + b2, s)
        assert _relerr(x12, x1 + x2) < 1e-13               # linear in b


def test_grid_transpose_is_equivariant():
    nx, ny = 8, 5
    a = W.random_grid_5pt(nx, ny, W.rng(408, 0), one_way=0.1)
    b = W.rng(408, 1).uniform(-1, 1, a.n)
    A = W.csr_to_dense(a)
    # relabel node (x, y) -> (y, x): rows become columns of the new grid
    p = np.array([x * ny + y for y in range(ny) for x in range(nx)])
    At = np.zeros_like(A)
    At[np.ix_(p, p)] = A
    bt = np.zeros_like(b)
    bt[p] = b
    rg, rgt = _lines(a, nx, ny), _lines(W.csr_from_dense(At), ny, nx)
    for s in (2, 3, 5):
        # the message state is equivariant (the read-off is not: it takes the column
        # solution, and columns become rows)
        _, lam, m = RG.run(rg, b, s)
        _, lamt, mt = RG.run(rgt, bt, s)
        assert _relerr(RG.readoff(rgt, bt, lamt, mt)[p], RG.readoff(rg, b, lam, m)) < 1e-13


# --------------------------------------------------------------------------------------
# precomputed precision messages and the smoother
# --------------------------------------------------------------------------------------

def test_precomputed_lambda_matches_the_joint_limit():
    nx, ny = 9, 8
    a = W.random_grid_5pt(nx, ny, W.rng(409, 0), one_way=0.1, flip=0.1)
    b = W.rng(409, 1).uniform(-1, 1, a.n)
    rg = _lines(a, nx, ny)
    lam, invs, ls = RG.lambda_phase(rg, 1e-14, 2000)
    assert ls < 2000
    _, lam_j, _ = RG.run(rg, np.zeros(a.n), ls + 40)
    assert max(np.abs(u - v).max() for u, v in zip(lam, lam_j)) < 1e-13
    x, st, _, _ = RG.solve(rg, b, 1e-13, 5000, precomp=(lam, invs))
    assert st == RG.OK
    assert _relerr(x, np.linalg.solve(W.csr_to_dense(a), b)) < 1e-11


def test_smoother_first_read_off_is_jacobi_and_a_line_is_solved_by_two():
    nx, ny = 11, 1
    a = W.random_grid_5pt(nx, ny, W.rng(410, 0), flip=0.2)
    A = W.csr_to_dense(a)
    r = W.rng(410, 1)
    b, x0 = r.uniform(-1, 1, a.n), r.uniform(-1, 1, a.n)
    rg = _lines(a, nx, ny)
    x1 = RG.smooth(rg, b, x0, 1)
    assert _relerr(x1, x0 + (b - A @ x0) / np.diag(A)) < 1e-15
    x2 = RG.smooth(rg, b, x0, 2)
    assert _relerr(x2, np.linalg.solve(A, b)) < 1e-13


def test_cover_check_rejects_bad_partitions():
    a = W.random_grid_5pt(4, 4, W.rng(411, 0))
    with pytest.raises(ValueError):
        RG.RegionGraph(a, RG.grid_lines(4, 4)[:4])                  # columns missing
    with pytest.raises(ValueError):
        RG.RegionGraph(a, RG.grid_lines(4, 4) + RG.grid_lines(4, 4)[:1])   # a row twice


# --------------------------------------------------------------------------------------
# the pins catch plausible mistakes (planted in a copy of the sweep, on the CPU)
# --------------------------------------------------------------------------------------

def _mutated_sweep(kind):
    def sweep(rg, b, lam, m, lam_fixed=None, groups=None):
        b = np.asarray(b, dtype=np.float64)
        tl, tm = RG._totals(rg, lam, m)
        x = (b + tm) / (rg.diag + tl)
        ln, mn, xr = [], [], []
        for k, r in enumerate(rg.regions):
            other_l, other_m = tl[r] - lam[k], tm[r] - m[k]
            if kind == "own_message_kept":          # region's own message not excluded
                other_l, other_m = tl[r], tm[r]
            inv = np.linalg.inv(rg.blocks[k] + np.diag(other_l))
            b0 = b[r] + (0 * other_m if kind == "no_mean_in" else other_m)
            xl = inv @ b0
            s = 1.0 / np.diag(inv)
            dd = 0.0 if kind == "diag_not_removed" else rg.diag[r]
            ln.append(s - dd - other_l)
            mn.append(s * xl - b[r] - other_m)
            if kind == "transposed_block":          # transposed operand
                inv = np.linalg.inv(rg.blocks[k].T + np.diag(other_l))
                s = 1.0 / np.diag(inv)
                ln[-1] = s - rg.diag[r] - other_l
                mn[-1] = s * (inv @ b0) - b[r] - other_m
            xr.append(xl)
        return x, xr, ln, mn
    return sweep


@pytest.mark.parametrize("kind", ["own_message_kept", "no_mean_in", "diag_not_removed",
                                  "transposed_block"])
def test_pins_detect_planted_mistakes(kind, monkeypatch):
    monkeypatch.setattr(RG, "sweep", _mutated_sweep(kind))
    failures = 0
    with np.errstate(all="ignore"):
        try:
            failures += not (_bethe_vs_gabp(W.random_grid_5pt(4, 3, W.rng(412, 0),
                                                               one_way=0.3), np.ones(12), 4)
                             < 1e-13)
        except Exception:
            failures += 1
        nx = 13
        a = W.random_grid_5pt(nx, 1, W.rng(412, 1), one_way=0.2)
        b = W.rng(412, 2).uniform(-1, 1, nx)
        x2, _, _ = RG.run(_lines(a, nx, 1), b, 2)
        failures += not (_relerr(x2, np.linalg.solve(W.csr_to_dense(a), b)) < 1e-13)
    assert failures >= 1, f"planted mistake {kind} passed every pin"


@pytest.mark.parametrize("mode", ["precomp", "joint"])
def test_rows_then_columns_smoother_in_a_v_cycle(mode):
    # soft: the grouped line smoother gives a contracting V(2,2) cycle on Poisson, while
    # the flood line smoother (like flood point GaBP, Sec. 4.1) does not smooth well
    from oracle import mg as MG
    csrs = W.mg_hierarchy(5, kx=1.0, ky=1.0, peclet=0.0)
    b = W.rng(415, 0).uniform(-1, 1, csrs[0].n)
    h = MG.Hierarchy(csrs, smoother="gabp", nu1=2, nu2=2, gabp_mode=mode,
                     schedule="lines_alt")
    _, hist = h.solve(b, 1e-8, 30)
    assert hist[-1] <= 1e-8 and len(hist) <= 20


def test_unplanted_copy_passes_the_pins(monkeypatch):
    """The copy of the region sweep the mistakes go into passes both pins with nothing
    planted, so each failure above comes from its mistake."""
    monkeypatch.setattr(RG, "sweep", _mutated_sweep("none"))
    assert _bethe_vs_gabp(W.random_grid_5pt(4, 3, W.rng(412, 0), one_way=0.3),
                          np.ones(12), 4) < 1e-13
    nx = 13
    a = W.random_grid_5pt(nx, 1, W.rng(412, 1), one_way=0.2)
    b = W.rng(412, 2).uniform(-1, 1, nx)
    x2, _, _ = RG.run(_lines(a, nx, 1), b, 2)
    assert _relerr(x2, np.linalg.solve(W.csr_to_dense(a), b)) < 1e-13
