"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

FP64 sweeps must match the oracle to 1e-12 relative (max-norm) after the same number of
sweeps; converged solves must reach the dense solution. Inputs are seeded and synthetic
(upwind convection-diffusion grids, random walk-summable and tree matrices), sized so the
oracle finishes in seconds while spanning several 64-row slices and a ragged tail.
"""
import numpy as np
import pytest

from conftest import golden
from oracle import adjoint as AD
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
    x = np.asarray(x)
    y = np.asarray(y)
    return float(np.abs(x - y).max() / max(np.abs(y).max(), 1e-300))


def _cases():
    out = {}
    a, b = W.small_upwind(32)
    out["upwind32"] = (a, b, None)
    r = W.rng(300, 0)
    a = W.random_walk_summable(200, 0.03, r)               # structurally nonsymmetric, ragged
    out["walk200"] = (a, r.uniform(-1, 1, a.n), None)
    a = W.random_tridiagonal(130, W.rng(300, 1))
    out["tridiag130"] = (a, W.rng(300, 2).uniform(-1, 1, a.n), None)
    a, _ = W.random_tree(150, W.rng(300, 3), one_way=0.3)
    out["tree150"] = (a, W.rng(300, 4).uniform(-1, 1, a.n), None)
    a, b = W.precision_at_scale(45)
    out["field45"] = (a, b, None)
    a = W.csr_from_dense(np.array([[2.5]]))
    out["n1"] = (a, np.array([0.7]), None)
    a, b = W.small_upwind(9)                                # n = 81: one slice + tail
    out["upwind9"] = (a, b, None)
    return out


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_joint_sweeps_match_oracle(B, name):
    a, b, _ = CASES[name]
    s = B.Solver.from_csr(a)
    g = G.Graph.from_csr(a)
    bt = _cuda(b)
    for sweeps in (1, 2, 3, 10, 100):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        xo, _, _ = G.run(g, b, sweeps)
        assert _rel_inf(x, xo) <= TOL, (name, sweeps)


@pytest.mark.parametrize("name", ["upwind32", "walk200", "field45", "tree150"])
def test_precomp_sweeps_match_oracle(B, name):
    a, b, _ = CASES[name]
    L = 40
    s = B.Solver.from_csr(a, mode="precomp", tol_lambda=0.0, max_lambda_sweeps=L)
    assert s.precompute_lambda() == L
    g = G.Graph.from_csr(a)
    Lt, S, k = G.lambda_phase(g, 0.0, L)
    bt = _cuda(b)
    for sweeps in (1, 2, 5, 50):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        m = np.zeros(g.E)
        for _ in range(sweeps):
            xo, m = G.msweep(g, b, Lt, S, m)
        assert _rel_inf(x, xo) <= TOL, (name, sweeps)


@pytest.mark.parametrize("mode", ["joint", "precomp"])
def test_redblack_sweeps_match_oracle(B, mode):
    n = 24
    a, b = W.small_upwind(n)
    colour = G.grid_colour(n)
    kw = dict(mode=mode, schedule="redblack")
    if mode == "precomp":
        kw.update(tol_lambda=0.0, max_lambda_sweeps=30)
    s = B.Solver.from_csr(a, colour=colour, **kw)
    g = G.Graph.from_csr(a)
    lam = None
    if mode == "precomp":
        Lt, S, _ = G.lambda_phase(g, 0.0, 30)
        lam = (Lt, S)
    bt = _cuda(b)
    for sweeps in (1, 2, 7, 40):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        Lt0 = np.zeros(g.E) if lam is None else lam[0]
        m = np.zeros(g.E)
        for _ in range(sweeps):
            xo, Lt0, m = G.sweep_coloured(g, b, Lt0, m, colour, lambda_fixed=lam)
        assert _rel_inf(x, xo) <= TOL, (mode, sweeps)


@pytest.mark.parametrize("mode", ["joint", "precomp"])
def test_redblack_class_relative_reverse_deltas(B, monkeypatch, mode):
    """Two colour classes on a 191 x 193 grid (36,863 rows, one-way and sign-flipped
    couplings): a slot and its reverse lie in different classes, tens of thousands of slots
    apart, so the 2-byte reverse deltas are taken from the other class's first slot, with a
    marker for padding slots (their own reverse). Sweeps match the oracle, and with every
    output buffer poisoned first the results are the same bits (every slot read was
    written)."""
    nx, ny = 191, 193
    a = W.random_grid_5pt(nx, ny, W.rng(320, 0), one_way=0.15, flip=0.2)
    b = W.rng(320, 1).uniform(-1, 1, a.n)
    idx = np.arange(a.n)
    colour = ((idx % nx + idx // nx) % 2).astype(np.uint8)
    kw = dict(mode=mode, schedule="redblack")
    if mode == "precomp":
        kw.update(tol_lambda=0.0, max_lambda_sweeps=30)
    s = B.Solver.from_csr(a, colour=colour, **kw)
    assert s.layout_info()["rev_bytes"] == 2
    g = G.Graph.from_csr(a)
    lam = None
    if mode == "precomp":
        Lt, S, _ = G.lambda_phase(g, 0.0, 30)
        lam = (Lt, S)
    bt = _cuda(b)
    for sweeps in (1, 2, 5):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        Lt0 = np.zeros(g.E) if lam is None else lam[0]
        m = np.zeros(g.E)
        for _ in range(sweeps):
            xo, Lt0, m = G.sweep_coloured(g, b, Lt0, m, colour, lambda_fixed=lam)
        assert _rel_inf(x, xo) <= TOL, (mode, sweeps)
    monkeypatch.setenv("GABP_FAULT_INJECT", "poison-outputs")
    poisoned = B.Solver.from_csr(a, colour=colour, **kw)
    monkeypatch.delenv("GABP_FAULT_INJECT")
    for tr in (False, True):
        want = s.sweeps(bt, 6, transposed=tr).cpu().numpy()
        got = poisoned.sweeps(bt, 6, transposed=tr).cpu().numpy()
        assert np.all(np.isfinite(got)) and np.array_equal(got, want), tr


def test_redblack_rejects_improper_colouring(B):
    a, _ = W.small_upwind(8)
    with pytest.raises(B.GaBPError) as e:
        B.Solver.from_csr(a, colour=np.zeros(64, np.uint8), schedule="redblack")
    assert e.value.status == B.EINVAL
    # the red-black colouring is not proper for a 9-point stencil; colours stop at 7
    m, _, _ = W.sec5_problem("mixed_derivative", 8, eps=0.01)
    with pytest.raises(B.GaBPError) as e:
        B.Solver.from_csr(m, colour=G.grid_colour(8), schedule="redblack")
    assert e.value.status == B.EINVAL
    with pytest.raises(B.GaBPError) as e:
        B.Solver.from_csr(a, colour=np.full(64, 8, np.uint8), schedule="redblack")
    assert e.value.status == B.EINVAL


@pytest.mark.parametrize("mode", ["joint", "precomp"])
@pytest.mark.parametrize("n", [31, 45])
def test_four_colour_sweeps_on_a_nine_point_grid_match_oracle(B, mode, n):
    # the paper's 4-colour GaBP: colour classes (ix mod 2) + 2 (iy mod 2) in turn, on a
    # dominant random 9-point operator (GaBP alone diverges on the mixed-derivative one,
    # where only the first few sweeps are comparable; see below)
    a = W.random_grid_9pt(n, n, W.rng(309, n))
    b = W.rng(309, 1).uniform(-1, 1, a.n)
    colour = G.grid_colour4(n)
    kw = dict(mode=mode, schedule="redblack")
    if mode == "precomp":
        kw.update(tol_lambda=0.0, max_lambda_sweeps=30)
    s = B.Solver.from_csr(a, colour=colour, **kw)
    g = G.Graph.from_csr(a)
    lam = None
    if mode == "precomp":
        Lt, S, _ = G.lambda_phase(g, 0.0, 30)
        lam = (Lt, S)
    for sweeps in (1, 2, 7, 30):
        x = s.sweeps(_cuda(b), sweeps).cpu().numpy()
        Lt0 = np.zeros(g.E) if lam is None else lam[0]
        m = np.zeros(g.E)
        for _ in range(sweeps):
            xo, Lt0, m = G.sweep_coloured(g, b, Lt0, m, colour, lambda_fixed=lam)
        assert _rel_inf(x, xo) <= TOL, (mode, n, sweeps)


def _greedy_colouring(a, skip=None):
    """Greedy proper colouring of the symmetrised pattern (smallest free colour, row order);
    `skip`: a colour value left unused (an empty class)."""
    nb = [set() for _ in range(a.n)]
    for i in range(a.n):
        for c in a.col[a.rowptr[i]:a.rowptr[i + 1]]:
            if c != i:
                nb[i].add(int(c))
                nb[int(c)].add(i)
    col = np.full(a.n, -1)
    for j in range(a.n):
        used = {col[k] for k in nb[j] if col[k] >= 0}
        c = 0
        while c in used or c == skip:
            c += 1
        col[j] = c
    return col.astype(np.uint8)


@pytest.mark.parametrize("case", ["walk200_8colours", "sparse3000_5colours_one_empty"])
@pytest.mark.parametrize("mode", ["joint", "precomp"])
def test_many_colour_classes_match_oracle(B, case, mode):
    """Coloured sweeps with up to 8 uneven colour classes (padding lanes after every class,
    and an empty class) against the coloured oracle."""
    if case.startswith("walk200"):
        a, b, _ = CASES["walk200"]
        colour = _greedy_colouring(a)
    else:
        a = W.random_sparse_dominant(3000, 2, W.rng(307, 0))
        b = W.rng(307, 1).uniform(-1, 1, a.n)
        colour = _greedy_colouring(a, skip=2)
    assert colour.max() < 8
    kw = dict(mode=mode, schedule="redblack")
    lam = None
    g = G.Graph.from_csr(a)
    if mode == "precomp":
        kw.update(tol_lambda=0.0, max_lambda_sweeps=40)
        Lt, S, _ = G.lambda_phase(g, 0.0, 40)
        lam = (Lt, S)
    s = B.Solver.from_csr(a, colour=colour, **kw)
    bt = _cuda(b)
    for sweeps in (1, 2, 5):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        Lt0, m = np.zeros(g.E), np.zeros(g.E)
        for _ in range(sweeps):
            xo, Lt0, m = G.sweep_coloured(g, b, Lt0, m, colour, lambda_fixed=lam)
        assert _rel_inf(x, xo) < TOL, (case, mode, sweeps)


def test_four_colour_sweeps_on_the_mixed_derivative_problem(B):
    a, b, _ = W.sec5_problem("mixed_derivative", 31, eps=0.01)
    colour = G.grid_colour4(31)
    s = B.Solver.from_csr(a, colour=colour, schedule="redblack")
    g = G.Graph.from_csr(a)
    for sweeps in (1, 2, 5):
        x = s.sweeps(_cuda(b), sweeps).cpu().numpy()
        Lt0, m = np.zeros(g.E), np.zeros(g.E)
        for _ in range(sweeps):
            xo, Lt0, m = G.sweep_coloured(g, b, Lt0, m, colour)
        assert _rel_inf(x, xo) <= TOL, sweeps


@pytest.mark.parametrize("mode", ["joint", "precomp"])
def test_solve_reaches_dense_solution(B, mode):
    a, b, _ = CASES["upwind32"]
    s = B.Solver.from_csr(a, mode=mode, check_every=8)
    x, info = s.solve(_cuda(b), 1e-13, 20000)
    assert info.status == B.OK and info.rel_res2 <= 1e-13
    xs = np.linalg.solve(W.csr_to_dense(a), b)
    assert _rel_inf(x.cpu().numpy(), xs) <= 1e-10
    # the oracle needs the same number of sweeps up to one check interval
    if mode == "joint":
        _, oinfo, _, _ = G.solve(G.Graph.from_csr(a), b, 1e-13, 20000, check_every=8)
        assert abs(oinfo.sweeps - info.sweeps) <= 8


def test_ir_fp32_messages_reach_fp64_accuracy(B):
    for name in ("upwind32", "field45"):
        a, b, _ = CASES[name]
        s = B.Solver.from_csr(a, precision="f32_ir", check_every=16, tol_lambda=1e-12)
        x, info = s.solve(_cuda(b), 1e-12, 200000)
        assert info.status == B.OK, (name, info)
        assert info.rel_res2 <= 1e-12 and info.outer_iters >= 2
        xs = np.linalg.solve(W.csr_to_dense(a), b)
        assert _rel_inf(x.cpu().numpy(), xs) <= 1e-8, name


@pytest.mark.parametrize("name", ["upwind32", "walk200", "tree150"])
def test_transposed_sweeps_match_oracle_on_AT(B, name):
    a, b, _ = CASES[name]
    s = B.Solver.from_csr(a)
    gt = G.Graph.from_csr(a).transposed()
    bt = _cuda(b)
    for sweeps in (1, 3, 30):
        x = s.sweeps(bt, sweeps, transposed=True).cpu().numpy()
        xo, _, _ = G.run(gt, b, sweeps)
        assert _rel_inf(x, xo) <= TOL


def test_transposed_solve(B):
    a, b, _ = CASES["field45"]
    s = B.Solver.from_csr(a, mode="precomp")
    lam, info = s.solve_transposed(_cuda(b), 1e-13, 50000)
    assert info.status == B.OK
    ls = np.linalg.solve(W.csr_to_dense(a).T, b)
    assert _rel_inf(lam.cpu().numpy(), ls) <= 1e-10


@pytest.mark.parametrize("mode", ["joint", "precomp", "seq"])
@pytest.mark.parametrize("schedule", ["flood", "redblack"])
def test_smoother_matches_oracle(B, mode, schedule):
    """Algorithm 3 from zero messages; with the per-sweep precomputed precision messages
    (seq) the oracle's joint smoother is the reference (the two are the same iterates)."""
    n = 20
    a, b = W.small_upwind(n)
    g = G.Graph.from_csr(a)
    col = G.grid_colour(n) if schedule == "redblack" else None
    kw = dict(mode=mode, schedule=schedule)
    lam = None
    if mode == "precomp":
        kw.update(tol_lambda=0.0, max_lambda_sweeps=25)
        Lt, S, _ = G.lambda_phase(g, 0.0, 25)
        lam = (Lt, S)
    s = B.Solver.from_csr(a, colour=col, **kw)
    x0 = W.rng(301, 0).uniform(-1, 1, a.n)
    xg = _cuda(x0)
    bt = _cuda(b)
    xo = x0.copy()
    for mu in (1, 2, 3, 2, 5):
        s.smooth(bt, xg, mu)
        xo = G.smooth(g, b, xo, mu, lam=lam) if col is None else \
            G.smooth_coloured(g, b, xo, mu, col, lam=lam)
        assert _rel_inf(xg.cpu().numpy(), xo) <= TOL, (mode, schedule, mu)


@pytest.mark.parametrize("schedule", ["flood", "redblack"])
def test_seq_fp32_smoother_is_the_joint_smoother_to_fp32_rounding(B, schedule):
    """FP32 mean messages with the per-sweep precision messages rounded once to FP32: the
    joint FP64 smoother's iterates to FP32 rounding (a few ulps per sweep)."""
    n = 24
    a, b = W.small_upwind(n)
    g = G.Graph.from_csr(a)
    col = G.grid_colour(n) if schedule == "redblack" else None
    s = B.Solver.from_csr(a, colour=col, mode="seq", precision="f32_ir", schedule=schedule)
    x0 = W.rng(302, 0).uniform(-1, 1, a.n)
    for mu in (1, 2, 4):
        xg = _cuda(x0)
        s.smooth(_cuda(b), xg, mu)
        xo = G.smooth(g, b, x0, mu) if col is None else G.smooth_coloured(g, b, x0, mu, col)
        # the correction e^mu carries the FP32 error, relative to its own size
        err = np.abs(xg.cpu().numpy() - xo).max() / np.abs(xo - x0).max()
        assert err <= 2e-6 * (1 + mu), (schedule, mu, err)


@pytest.mark.parametrize("name", ["upwind32", "walk200", "tree150", "upwind9"])
def test_seq_sweeps_match_joint_oracle(B, name):
    """gabp_sweeps in the per-sweep precomputed mode, from a reset and continued without
    one (the stored sequence grows on demand), against the oracle's joint iteration."""
    a, b, _ = CASES[name]
    s = B.Solver.from_csr(a, mode="seq")
    g = G.Graph.from_csr(a)
    bt = _cuda(b)
    for sweeps in (1, 2, 3, 10):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        xo, _, _ = G.run(g, b, sweeps)
        assert _rel_inf(x, xo) <= TOL, (name, sweeps)
    x = s.sweeps(bt, 4, reset=False).cpu().numpy()      # sweeps 11..14
    xo, _, _ = G.run(g, b, 14)
    assert _rel_inf(x, xo) <= TOL, name


def test_seq_mode_rejects_solves(B):
    a, b = W.small_upwind(8)
    s = B.Solver.from_csr(a, mode="seq")
    with pytest.raises(B.GaBPError) as e:
        s.solve(_cuda(b), 1e-8, 100)
    assert e.value.status == B.ENOTSUPP
    with pytest.raises(B.GaBPError) as e:
        B.Solver.from_csr(a, mode="seq", schedule="lines", grid=(8, 8))
    assert e.value.status == B.ENOTSUPP


def _oracle_edges(a):
    """CSR positions of the oracle's edges (off-diagonal entries with A_ij != 0), in the
    oracle's edge order."""
    rows = a.row_of_nnz()
    return np.nonzero((rows != a.col) & (a.val != 0.0))[0]


def _rel_msgs(got, want):
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


@pytest.mark.parametrize("name", list(CASES))
def test_joint_messages_match_oracle(B, name):
    """The messages themselves (Lt_ji, m_ji of eq. nonsymmetric_GaBP_rules), not only the
    read-offs, after 1, 2, 3 and 10 sweeps."""
    a, b, _ = CASES[name]
    s = B.Solver.from_csr(a)
    g = G.Graph.from_csr(a)
    idx = _oracle_edges(a)
    assert len(idx) == g.E
    bt = _cuda(b)
    for sweeps in (1, 2, 3, 10):
        s.sweeps(bt, sweeps)
        lam, msg = (t.cpu().numpy() for t in s.messages())
        _, Lt, m = G.run(g, b, sweeps)
        if g.E:
            assert _rel_msgs(lam[idx], Lt) <= TOL, (name, sweeps)
            assert _rel_msgs(msg[idx], m) <= TOL, (name, sweeps)
        rest = np.setdiff1d(np.arange(a.nnz), idx)
        assert np.all(lam[rest] == 0.0) and np.all(msg[rest] == 0.0)


@pytest.mark.parametrize("mode", ["precomp", "seq"])
@pytest.mark.parametrize("schedule", ["flood", "redblack"])
def test_precomputed_messages_match_oracle(B, mode, schedule):
    n = 24
    a, b = W.small_upwind(n)
    g = G.Graph.from_csr(a)
    col = G.grid_colour(n) if schedule == "redblack" else None
    kw = dict(mode=mode, schedule=schedule)
    if mode == "precomp":
        kw.update(tol_lambda=0.0, max_lambda_sweeps=30)
    s = B.Solver.from_csr(a, colour=col, **kw)
    idx = _oracle_edges(a)
    lamfix = None
    if mode == "precomp":
        Lt, S, _ = G.lambda_phase(g, 0.0, 30)
        lamfix = (Lt, S)
    bt = _cuda(b)
    for sweeps in (1, 2, 5):
        s.sweeps(bt, sweeps)
        lam, msg = (t.cpu().numpy() for t in s.messages())
        L0, m = (np.zeros(g.E) if lamfix is None else lamfix[0]), np.zeros(g.E)
        for _ in range(sweeps):
            if col is not None:
                _, L0, m = G.sweep_coloured(g, b, L0, m, col, lambda_fixed=lamfix)
            elif lamfix is None:
                _, L0, m, _, _ = G.sweep(g, b, L0, m)
            else:
                _, m = G.msweep(g, b, lamfix[0], lamfix[1], m)
        assert _rel_msgs(lam[idx], L0) <= TOL, (mode, schedule, sweeps)
        assert _rel_msgs(msg[idx], m) <= TOL, (mode, schedule, sweeps)


def test_residual_and_norms(B):
    a, b, _ = CASES["walk200"]
    s = B.Solver.from_csr(a)
    x = W.rng(302, 0).uniform(-1, 1, a.n)
    r, (n2, ninf, bn) = s.residual(_cuda(b), _cuda(x))
    ro = G.Graph.from_csr(a).residual(b, x)
    assert _rel_inf(r.cpu().numpy(), ro) <= 1e-14
    assert n2 == pytest.approx(np.linalg.norm(ro), rel=1e-13)
    assert ninf == pytest.approx(np.abs(ro).max(), rel=1e-14)
    assert bn == pytest.approx(np.linalg.norm(b), rel=1e-13)
    rt, _ = s.residual(_cuda(b), _cuda(x), transposed=True)
    assert _rel_inf(rt.cpu().numpy(), b - W.csr_to_dense(a).T @ x) <= 1e-14


def test_adjoint_scatter_matches_oracle(B):
    n = 16
    theta = W.theta_problem(n, 0)
    a, jptr, jnnz, jw = W.theta_jacobian(n, theta)
    s = B.Solver.from_csr(a)
    r = W.rng(303, 0)
    lam = r.uniform(-1, 1, a.n)
    x = r.uniform(-1, 1, a.n)
    Gd, dth = s.adjoint_scatter(_cuda(lam), _cuda(x),
                                jac=(torch.as_tensor(jptr).cuda(), torch.as_tensor(jnnz).cuda(),
                                     _cuda(jw)))
    Go = AD.nnz_gradient(a.row_of_nnz(), a.col, lam, x)
    assert np.array_equal(Gd.cpu().numpy(), Go)
    do = AD.reduce_to_params(Go, jptr, jnnz, jw)
    assert _rel_inf(dth.cpu().numpy(), do) <= 1e-14


def test_full_size_adjoint_scatter_matches_oracle(B):
    """The differentiation configuration's grid (1024 x 1024 cells, 5.2M stored entries,
    theta = per-cell log-diffusion): the entry gradient -lambda_i x_j equals the oracle's bit
    for bit and its reduction onto theta matches to 1e-14."""
    n = 1024
    theta = W.theta_problem(n, 0)
    a, jptr, jnnz, jw = W.theta_jacobian(n, theta)
    s = B.Solver.from_csr(a)
    r = W.rng(303, 1)
    lam = r.uniform(-1, 1, a.n)
    x = r.uniform(-1, 1, a.n)
    Gd, dth = s.adjoint_scatter(_cuda(lam), _cuda(x),
                                jac=(torch.as_tensor(jptr).cuda(), torch.as_tensor(jnnz).cuda(),
                                     _cuda(jw)))
    Go = AD.nnz_gradient(a.row_of_nnz(), a.col, lam, x)
    assert np.array_equal(Gd.cpu().numpy(), Go)
    do = AD.reduce_to_params(Go, jptr, jnnz, jw)
    assert _rel_inf(dth.cpu().numpy(), do) <= 1e-14


def test_checkpoint_resume_is_bitwise(B):
    a, b, _ = CASES["walk200"]
    s = B.Solver.from_csr(a)
    bt = _cuda(b)
    s.sweeps(bt, 7)
    blob = s.get_state()
    x1 = s.sweeps(bt, 5, reset=False).cpu().numpy()
    s.sweeps(bt, 3)                 # disturb the state
    s.set_state(blob)
    x2 = s.sweeps(bt, 5, reset=False).cpu().numpy()
    assert np.array_equal(x1, x2)
    x12 = s.sweeps(bt, 12).cpu().numpy()
    assert np.array_equal(x12, x1)   # 7 + 5 sweeps from zero, same bits


def test_checkpoint_rejects_another_layout_or_mode(B):
    """On a 32 x 32 grid the flood and the red-black layouts have the same padded slot count
    but different message positions: a blob of one must not load into the other, nor into
    a context of another mode or precision."""
    a, b, _ = CASES["upwind32"]
    bt = _cuda(b)
    flood = B.Solver.from_csr(a)
    rb = B.Solver.from_csr(a, colour=W.grid_colouring(32), schedule="redblack")
    assert flood.layout_info()["padded_slots"] == rb.layout_info()["padded_slots"]
    flood.sweeps(bt, 4)
    blob = flood.get_state()
    for other in (rb, B.Solver.from_csr(a, mode="seq"),
                  B.Solver.from_csr(a, mode="precomp", precision="f32_ir")):
        with pytest.raises(B.GaBPError) as e:
            other.set_state(blob)
        assert e.value.status == B.EINVAL
    B.Solver.from_csr(a).set_state(blob)                   # same layout and mode: accepted


def test_seq_checkpoint_resumes(B):
    """The per-sweep mode's checkpoint carries the sweep position: 4 sweeps, checkpoint,
    3 more equal 7 from zero messages (the stored sequence grows to 7 on demand)."""
    a, b, _ = CASES["walk200"]
    bt = _cuda(b)
    s = B.Solver.from_csr(a, mode="seq")
    s.sweeps(bt, 4)
    blob = s.get_state()
    r = B.Solver.from_csr(a, mode="seq")
    r.set_state(blob)
    x = r.sweeps(bt, 3, reset=False).cpu().numpy()
    assert np.array_equal(x, s.sweeps(bt, 7).cpu().numpy())
    xo, _, _ = G.run(G.Graph.from_csr(a), b, 7)
    assert _rel_inf(x, xo) <= TOL


@pytest.mark.parametrize("kw", [dict(mode="joint"),
                                dict(mode="joint", schedule="redblack"),
                                dict(mode="precomp", precision="f32_ir", tol_lambda=1e-10),
                                dict(mode="joint", schedule="lines_alt", grid=(32, 32)),
                                dict(mode="joint", schedule="lines", grid=(32, 32))])
def test_reset_state_is_zero_messages_everywhere(B, kw):
    """A reset marks the messages zero without clearing them; every reader agrees: the next
    sweeps (reset or not), a checkpoint taken in that state, and a context restored from it."""
    a, b, _ = CASES["upwind32"]
    if kw.get("schedule") == "redblack":
        kw = dict(kw, colour=W.grid_colouring(32))
    bt = _cuda(b)
    ref = B.Solver.from_csr(a, **kw)
    want = ref.sweeps(bt, 3).cpu().numpy()               # 3 sweeps from zero messages
    s = B.Solver.from_csr(a, **kw)
    s.sweeps(bt, 5)                                      # some non-zero message state
    s.autotune()                                         # leaves the messages reset
    blob = s.get_state()
    r = B.Solver.from_csr(a, **kw)
    r.sweeps(bt, 2)
    r.set_state(blob)
    assert np.array_equal(r.sweeps(bt, 3, reset=False).cpu().numpy(), want)
    assert np.array_equal(s.sweeps(bt, 3, reset=False).cpu().numpy(), want)
    assert np.array_equal(s.sweeps(bt, 3).cpu().numpy(), want)


def test_repeat_runs_are_bitwise_identical(B):
    a, b, _ = CASES["field45"]
    s = B.Solver.from_csr(a, check_every=4)
    bt = _cuda(b)
    x1, i1 = s.solve(bt, 1e-8, 400)
    x2, i2 = s.solve(bt, 1e-8, 400)
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert i1.rel_res2 == i2.rel_res2


def test_update_values_matches_fresh_setup(B):
    n = 20
    t0, t1 = W.theta_problem(n, 0), W.theta_problem(n, 1)
    a0 = W.theta_operator(n, t0)
    a1 = W.theta_operator(n, t1)
    assert np.array_equal(a0.col, a1.col)
    b = W.rng(304, 0).uniform(-1, 1, a0.n)
    s = B.Solver.from_csr(a0)
    s.update_values(_cuda(a1.val))
    fresh = B.Solver.from_csr(a1)
    bt = _cuda(b)
    assert np.array_equal(s.sweeps(bt, 9).cpu().numpy(), fresh.sweeps(bt, 9).cpu().numpy())
    bad = a1.val.copy()
    bad[a1.row_of_nnz() == a1.col] = 0.0
    with pytest.raises(B.GaBPError) as e:
        s.update_values(_cuda(bad))
    assert e.value.status == B.EZERODIAG


def test_failure_modes(B):
    # zero cavity precision: [[1, 1], [1, 1]] has Sigma_j - Lt_ij A_ij = 1 - 1 = 0 at sweep 2
    a = W.csr_from_dense(np.array([[1.0, 1.0], [1.0, 1.0]]))
    s = B.Solver.from_csr(a, check_every=1)
    with pytest.raises(B.GaBPError) as e:
        s.solve(_cuda([1.0, 2.0]), 1e-12, 10)
    assert e.value.status == B.ENUMERIC
    # the 7x7 example of Sec. 3.4 does not converge
    A = np.loadtxt(golden("paper_7x7.txt"), comments="#")
    s = B.Solver.from_csr(W.csr_from_dense(A), check_every=50)
    try:
        _, info = s.solve(_cuda(np.ones(7)), 1e-10, 2000)
        assert info.status == B.MAXSWEEPS
    except B.GaBPError as err:
        assert err.status == B.ENUMERIC
    # max_sweeps reached
    a, b, _ = CASES["upwind32"]
    s = B.Solver.from_csr(a, check_every=4)
    _, info = s.solve(_cuda(b), 1e-14, 8)
    assert info.status == B.MAXSWEEPS and info.sweeps == 8
    with pytest.raises(B.GaBPError):
        s.solve(_cuda(b), 1e-14, 0)


@pytest.mark.parametrize("kw,at", [(dict(mode="joint"), 8),
                                   (dict(mode="precomp", precision="f32_ir", tol_lambda=1e-10), 16),
                                   (dict(mode="joint", schedule="lines_alt", grid=(32, 32)), 8)])
def test_injected_nan_is_reported(B, monkeypatch, kw, at):
    """A NaN forced into the messages from the host (GABP_FAULT_INJECT) reaches the check
    that follows it and ends the solve with ENUMERIC; the checks before it stay finite."""
    a, b, _ = CASES["upwind32"]
    monkeypatch.setenv("GABP_FAULT_INJECT", f"nan@sweep:{at}")
    s = B.Solver.from_csr(a, check_every=4, **kw)
    monkeypatch.delenv("GABP_FAULT_INJECT")
    with pytest.raises(B.GaBPError) as e:
        s.solve(_cuda(b), 1e-14, 4000)
    assert e.value.status == B.ENUMERIC
    h = s.residual_history()
    assert len(h) >= 2 and np.isnan(h[-1]) and np.all(np.isfinite(h[:-1]))
    if "precision" not in kw:
        assert len(h) == at // 4 + 1                 # the block that starts at sweep `at`
    # injection happens once: the same context solves normally afterwards
    x, info = s.solve(_cuda(b), 1e-10, 40000)
    assert info.status == B.OK
    monkeypatch.setenv("GABP_FAULT_INJECT", "inf@7")
    with pytest.raises(B.GaBPError) as e:
        B.Solver.from_csr(a)
    assert e.value.status == B.EINVAL


@pytest.mark.parametrize("kw", [dict(mode="joint"),
                                dict(mode="precomp", precision="f64", tol_lambda=1e-12),
                                dict(mode="precomp", precision="f32_ir", tol_lambda=1e-10),
                                dict(mode="joint", schedule="lines", grid=(32, 32)),
                                dict(mode="precomp", precision="f32_ir", tol_lambda=1e-10,
                                     schedule="lines_alt", grid=(32, 32))])
def test_every_output_slot_is_written(B, monkeypatch, kw):
    """Race/coverage check: with every sweep's output buffers filled with NaN first
    (GABP_FAULT_INJECT=poison-outputs), sweeps and solves give the same bits as without."""
    a, b, _ = CASES["upwind32"]
    bt = _cuda(b)
    clean = B.Solver.from_csr(a, check_every=8, **kw)
    monkeypatch.setenv("GABP_FAULT_INJECT", "poison-outputs")
    poisoned = B.Solver.from_csr(a, check_every=8, **kw)
    monkeypatch.delenv("GABP_FAULT_INJECT")
    for tr in (False, True):
        want = clean.sweeps(bt, 9, transposed=tr).cpu().numpy()
        got = poisoned.sweeps(bt, 9, transposed=tr).cpu().numpy()
        assert np.all(np.isfinite(got)) and np.array_equal(got, want), tr
    xw, iw = clean.solve(bt, 1e-9, 40000)
    xg, ig = poisoned.solve(bt, 1e-9, 40000)
    assert ig.status == B.OK and ig.sweeps == iw.sweeps
    assert np.array_equal(xg.cpu().numpy(), xw.cpu().numpy())


@pytest.mark.parametrize("name", ["walk200", "tree150", "upwind9", "n1", "sparse20k"])
@pytest.mark.parametrize("mode", ["joint", "precomp"])
def test_every_output_slot_is_written_ragged(B, monkeypatch, name, mode):
    """The same check on ragged, one-way and tiny graphs (padding slots of short rows,
    missing reverses), and on long-range couplings that need the 4-byte reverse index."""
    if name == "sparse20k":
        a = W.random_sparse_dominant(20000, 3, W.rng(300, 9))
        b = W.rng(300, 10).uniform(-1, 1, a.n)
    else:
        a, b, _ = CASES[name]
    bt = _cuda(b)
    kw = dict(mode=mode, tol_lambda=0.0, max_lambda_sweeps=40)
    clean = B.Solver.from_csr(a, **kw)
    monkeypatch.setenv("GABP_FAULT_INJECT", "poison-outputs")
    poisoned = B.Solver.from_csr(a, **kw)
    monkeypatch.delenv("GABP_FAULT_INJECT")
    if name == "sparse20k":
        assert clean.layout_info()["rev_bytes"] == 4
    for k in (1, 2, 7):
        want = clean.sweeps(bt, k).cpu().numpy()
        got = poisoned.sweeps(bt, k).cpu().numpy()
        assert np.array_equal(got, want), k


def test_residual_history_records_every_check(B):
    a, b, _ = CASES["upwind32"]
    s = B.Solver.from_csr(a, check_every=8)
    x, info = s.solve(_cuda(b), 1e-10, 40000)
    h = s.residual_history()
    assert info.status == B.OK and len(h) == info.sweeps // 8
    assert h[-1] == info.rel_res2 and h[-1] <= 1e-10 and np.all(h[:-1] > 1e-10)
    s.solve(_cuda(b), 1e-3, 40000)                   # the next solve replaces the history
    assert len(s.residual_history()) < len(h)


def _ball(a, centre, radius):
    seen = {int(centre)}
    frontier = [int(centre)]
    for _ in range(radius):
        nxt = []
        for u in frontier:
            for c in a.col[a.rowptr[u]:a.rowptr[u + 1]]:
                if int(c) not in seen:
                    seen.add(int(c))
                    nxt.append(int(c))
        frontier = nxt
    return np.array(sorted(seen))


def test_full_size_sampled_parity(B):
    """2048 x 2048 variable-coefficient operator (4.19M unknowns) in the launch
    configuration the benchmark times: sampled read-offs after s sweeps equal the oracle run
    on the radius-s ball around each sample (x_j after s sweeps depends on nothing else),
    and the messages into each sample after s updates equal the oracle's on the radius
    s + 1 ball (a message i -> j depends on the radius-s ball around i)."""
    a, b = W.precision_at_scale(2048)
    s = B.Solver.from_csr(a)
    bt = _cuda(b)
    samples = W.rng(305, 0).choice(a.n, 48, replace=False)
    samples[0], samples[1], samples[2] = 0, a.n - 1, 2047    # corners
    for sweeps in (1, 2, 5, 12, 20):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        lam, msg = ((t.cpu().numpy() for t in s.messages()) if sweeps in (1, 5, 20)
                    else (None, None))
        for j in samples:
            sub_a, sub_b, nodes, sj = _ball_problem(a, b, j, sweeps)
            xo, _, _ = G.run(G.Graph.from_csr(sub_a), sub_b, sweeps)
            assert abs(x[j] - xo[sj]) <= TOL * max(abs(xo[sj]), 1e-300) + 1e-300, (j, sweeps)
            if lam is None:
                continue
            sub_a, sub_b, nodes, sj = _ball_problem(a, b, j, sweeps + 1)
            g = G.Graph.from_csr(sub_a)
            _, Lt, m = G.run(g, sub_b, sweeps)
            into = np.nonzero(g.dst == sj)[0]                    # oracle edges i -> j
            lo, hi = a.rowptr[j], a.rowptr[j + 1]
            off = np.nonzero(a.col[lo:hi] != j)[0] + lo          # CSR entries (j, i)
            assert len(into) == len(off)
            assert np.allclose(lam[off], Lt[into], rtol=TOL, atol=0), (j, sweeps)
            assert np.allclose(msg[off], m[into], rtol=TOL,
                               atol=TOL * np.abs(m[into]).max()), (j, sweeps)
    # property at full size: the residual of the 20-sweep read-off is finite and below that
    # of x = 0
    r, (n2, _, bn) = s.residual(bt, torch.as_tensor(x).cuda())
    assert np.isfinite(n2) and n2 < bn


def _ball_problem(a, b, j, radius):
    """The sub-system on the radius-`radius` graph ball around j (CSR, rhs, nodes, j's index)."""
    nodes = _ball(a, j, radius)
    rows = []
    for u in nodes:
        lo, hi = a.rowptr[u], a.rowptr[u + 1]
        keep = np.isin(a.col[lo:hi], nodes)
        rows.append((np.searchsorted(nodes, a.col[lo:hi][keep]), a.val[lo:hi][keep]))
    rp = np.zeros(len(nodes) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(c) for c, _ in rows])
    sub_a = W.CSR(len(nodes), rp, np.concatenate([c for c, _ in rows]).astype(np.int32),
                  np.concatenate([v for _, v in rows]))
    return sub_a, b[nodes], nodes, int(np.searchsorted(nodes, j))


def test_full_size_f32_sampled_parity(B):
    """The FP32 refinement inner kernel at 2048 x 2048 in its launch configuration: after
    K = 20 Lt sweeps and s FP32 mean sweeps, a read-off depends only on the graph ball of
    radius K + s + 1 around its node, so sampled read-offs are compared with the FP64
    oracle on that ball, to FP32 rounding."""
    a, b = W.precision_at_scale(2048)
    K = 20
    s = B.Solver.from_csr(a, mode="precomp", precision="f32_ir", tol_lambda=0.0,
                          max_lambda_sweeps=K)
    bt = _cuda(b)
    samples = W.rng(307, 2).choice(a.n, 6, replace=False)
    samples[0], samples[1] = 0, a.n - 1
    for sweeps in (1, 5):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        for j in samples:
            sub_a, sub_b, nodes, sj = _ball_problem(a, b, j, K + sweeps + 1)
            g = G.Graph.from_csr(sub_a)
            Lt, S, _ = G.lambda_phase(g, 0.0, K)
            m = np.zeros(g.E)
            for _ in range(sweeps):
                xo, m = G.msweep(g, sub_b, Lt, S, m)
            assert abs(x[j] - xo[sj]) <= 2e-6 * (1 + sweeps) * np.abs(xo).max(), (j, sweeps)


@pytest.mark.parametrize("op", ["upwind5_redblack", "grid9_colour4"])
def test_full_size_coloured_sampled_parity(B, op):
    """Coloured schedules at 2048 x 2048 in the launch configuration the coloured-sweep
    benchmark times (colour-major lanes, 2-byte class-relative reverse deltas for red-black,
    4-byte reverse index for four colours): sampled read-offs after s
    sweeps equal the coloured oracle on the graph ball of radius K s + 2 around each sample
    (within one sweep a message can cross at most K edges, one per colour class)."""
    n = 2048
    if op == "upwind5_redblack":
        a, b = W.precision_at_scale(n)
        colour = W.grid_colouring(n)
    else:
        a = W.random_grid_9pt(n, n, W.rng(6, 0))
        b = W.rng(6, 1).uniform(-1, 1, a.n)
        colour = W.grid_colouring4(n)
    K = int(colour.max()) + 1
    s = B.Solver.from_csr(a, colour=colour, schedule="redblack")
    # two classes: 2-byte deltas from the other class's first slot; four: 4-byte indices
    assert s.layout_info()["rev_bytes"] == (2 if K == 2 else 4)
    bt = _cuda(b)
    samples = W.rng(306, K).choice(a.n, 6, replace=False)
    samples[0], samples[1] = 0, a.n - 1
    for sweeps in (1, 3):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        for j in samples:
            sub_a, sub_b, nodes, sj = _ball_problem(a, b, j, K * sweeps + 2)
            g = G.Graph.from_csr(sub_a)
            Lt, m = np.zeros(g.E), np.zeros(g.E)
            for _ in range(sweeps):
                xo, Lt, m = G.sweep_coloured(g, sub_b, Lt, m, colour[nodes])
            assert abs(x[j] - xo[sj]) <= TOL * max(abs(xo[sj]), 1e-300) + 1e-300, (op, j, sweeps)


def test_f32_mean_sweeps_track_fp64_oracle(B):
    """FP32 mean-only sweeps (the refinement inner kernel) against the FP64 oracle: equal up
    to FP32 rounding, which grows at most linearly with the sweep count."""
    for name in ("upwind32", "field45", "walk200"):
        a, b, _ = CASES[name]
        s = B.Solver.from_csr(a, mode="precomp", precision="f32_ir", tol_lambda=0.0,
                              max_lambda_sweeps=40)
        g = G.Graph.from_csr(a)
        Lt, S, _ = G.lambda_phase(g, 0.0, 40)
        bt = _cuda(b)
        for sweeps in (1, 5, 50):
            x = s.sweeps(bt, sweeps).cpu().numpy()
            m = np.zeros(g.E)
            for _ in range(sweeps):
                xo, m = G.msweep(g, b, Lt, S, m)
            assert _rel_inf(x, xo) <= 2e-6 * (1 + sweeps), (name, sweeps)


@pytest.mark.parametrize("kw", [dict(mode="joint"), dict(mode="precomp"),
                                dict(mode="precomp", precision="f32_ir"),
                                dict(mode="joint", schedule="redblack")])
def test_graph_replays_match_eager(B, kw):
    """Recorded check blocks replayed several times, with eager work in between, give the
    eager result bit for bit."""
    n = 24
    a, b = W.small_upwind(n)
    colour = G.grid_colour(n) if kw.get("schedule") == "redblack" else None
    eager = B.Solver.from_csr(a, colour=colour, check_every=8, use_graphs=False, **kw)
    graph = B.Solver.from_csr(a, colour=colour, check_every=8, use_graphs=True, **kw)
    bt = _cuda(b)
    xe, ie = eager.solve(bt, 1e-11, 20000)
    xe = xe.cpu().numpy()
    for rep in range(3):
        xg, ig = graph.solve(bt, 1e-11, 20000)
        assert np.array_equal(xg.cpu().numpy(), xe), rep
        assert ig.sweeps == ie.sweeps and ig.rel_res2 == ie.rel_res2
        eager.sweeps(bt, 5)                          # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("kw", [dict(mode="joint"), dict(mode="precomp", tol_lambda=1e-12),
                                dict(mode="precomp", precision="f32_ir", tol_lambda=1e-10)])
def test_recorded_solves_follow_new_values_and_tensors(B, kw):
    """A recorded solve reads the coefficients in place and stages b and x through the
    context, so it stays correct when the values change and when every call passes fresh
    tensors (the autograd pattern)."""
    n = 20
    ops = [W.theta_operator(n, W.theta_problem(n, q)) for q in range(3)]
    eager = B.Solver.from_csr(ops[0], check_every=8, use_graphs=False, **kw)
    graph = B.Solver.from_csr(ops[0], check_every=8, use_graphs=True, **kw)
    for q, a in enumerate(ops + ops[:1]):
        b = W.rng(305, q).uniform(-1, 1, a.n)
        for s in (eager, graph):
            s.update_values(_cuda(a.val))
        xe, ie = eager.solve(_cuda(b), 1e-10, 200000)
        xg, ig = graph.solve(_cuda(b), 1e-10, 200000)
        assert np.array_equal(xg.cpu().numpy(), xe.cpu().numpy()), q
        assert ig.sweeps == ie.sweeps, q
        xt, _ = graph.solve_transposed(_cuda(b), 1e-10, 200000)
        At = W.csr_to_dense(a).T
        assert np.abs(At @ xt.cpu().numpy() - b).max() < 1e-8 * np.abs(b).max() * 10, q


def test_batched_graph_replays_match_eager(B):
    fam = W.batch_family(nsys=5, nrhs=2, side_lo=8, side_hi=24, seed=33)
    systems = [x for x, _ in fam]
    rhs = np.stack([np.concatenate([bb[q] for _, bb in fam]) for q in range(2)])
    Bt = torch.as_tensor(rhs).cuda()
    res = []
    for graphs in (False, True, True, True):
        bs = B.BatchSolver(systems, nrhs=2, mode="precomp", precision="f32_ir",
                           check_every=16, tol_lambda=1e-8, use_graphs=graphs)
        X, infos = bs.solve(Bt, 1e-10, 200000)
        X2, _ = bs.solve(Bt, 1e-10, 200000)          # replay on the same context
        res.append((X.cpu().numpy(), X2.cpu().numpy(), [i.sweeps for i in infos]))
    for X, X2, sw in res[1:]:
        assert np.array_equal(X, res[0][0]) and np.array_equal(X2, res[0][0])
        assert sw == res[0][2]


@pytest.mark.parametrize("kw", [dict(mode="joint"), dict(mode="precomp", precision="f32_ir")])
def test_autotune_keeps_results_correct(B, kw):
    a, b, _ = CASES["field45"]
    s = B.Solver.from_csr(a, tol_lambda=1e-10, **kw)
    t = s.autotune()
    assert t["check_every"] in (8, 16, 32, 64, 128, 256) and t["stream_hints"] in (0, 1)
    assert t["block"] in (64, 128, 256)
    assert s.autotune() == t                       # cached
    x, info = s.solve(_cuda(b), 1e-11, 200000)
    assert info.status == B.OK and info.sweeps % t["check_every"] == 0 or info.outer_iters > 0
    xs = np.linalg.solve(W.csr_to_dense(a), b)
    assert _rel_inf(x.cpu().numpy(), xs) <= 1e-8


@pytest.mark.parametrize("schedule", ["flood", "redblack"])
def test_workgroup_sizes_agree(B, schedule):
    """The sweep kernels give the same bits at every workgroup size the autotuner picks
    from (one, two or four 64-row slices per workgroup)."""
    a, b, _ = CASES["upwind32"]
    col = G.grid_colour(32) if schedule == "redblack" else None
    outs = []
    for blk in (64, 128, 256):
        for kw in (dict(mode="joint"), dict(mode="seq"), dict(mode="precomp", precision="f32_ir")):
            s = B.Solver.from_csr(a, colour=col, schedule=schedule, block=blk, **kw)
            outs.append((blk, str(kw), s.sweeps(_cuda(b), 9).cpu().numpy()))
    for blk, kw, x in outs:
        ref = next(o for o in outs if o[1] == kw)[2]
        assert np.array_equal(x, ref), (blk, kw)
    with pytest.raises(B.GaBPError):
        B.Solver.from_csr(a, block=96)


def test_stream_hint_variants_agree(B):
    """Both streaming variants of the sweep kernels compute the same bits."""
    a, b, _ = CASES["upwind32"]
    outs = []
    for trial in range(2):
        s = B.Solver.from_csr(a, mode="joint")
        if trial:
            s.autotune()
        outs.append(s.sweeps(_cuda(b), 37).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("density,kw", [(0.3, dict(mode="joint")),          # two-pass
                                        (0.3, dict(mode="precomp", tol_lambda=0.0,
                                                   max_lambda_sweeps=30)),
                                        (0.02, dict(mode="joint")),           # width <= 16
                                        (0.02, dict(mode="precomp", precision="f64",
                                                    tol_lambda=0.0, max_lambda_sweeps=30))])
def test_wide_rows_two_pass_kernels(B, density, kw):
    """Rows with more than 16 (and more than 8) neighbours take the wider register or the
    two-pass kernel variants; they must agree with the oracle like the narrow ones."""
    r = W.rng(310, int(density * 100))
    a = W.random_walk_summable(150, density, r)
    widths = np.diff(a.rowptr)
    assert widths.max() > 5
    b = r.uniform(-1, 1, a.n)
    s = B.Solver.from_csr(a, **kw)
    g = G.Graph.from_csr(a)
    bt = _cuda(b)
    lam = G.lambda_phase(g, 0.0, 30) if kw["mode"] == "precomp" else None
    for sweeps in (1, 4, 25):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        if lam is None:
            xo, _, _ = G.run(g, b, sweeps)
        else:
            m = np.zeros(g.E)
            for _ in range(sweeps):
                xo, m = G.msweep(g, b, lam[0], lam[1], m)
        assert _rel_inf(x, xo) <= TOL, sweeps
    xr = r.uniform(-1, 1, a.n)          # residual kernel on wide rows, at a non-solution
    r_, _ = s.residual(bt, _cuda(xr))
    assert _rel_inf(r_.cpu().numpy(), g.residual(b, xr)) <= 1e-13


def test_long_range_pattern_int32_reverse_index(B):
    """Long-range couplings put reverse slots far apart: the 4-byte reverse index is used and
    the sweeps still match the oracle; grid matrices get the 2-byte deltas."""
    r = W.rng(311, 0)
    a = W.random_sparse_dominant(40000, 3, r)
    b = r.uniform(-1, 1, a.n)
    s = B.Solver.from_csr(a)
    assert s.layout_info()["rev_bytes"] == 4
    g = G.Graph.from_csr(a)
    bt = _cuda(b)
    for sweeps in (1, 3, 20):
        x = s.sweeps(bt, sweeps).cpu().numpy()
        xo, _, _ = G.run(g, b, sweeps)
        assert _rel_inf(x, xo) <= TOL
    p = B.Solver.from_csr(a, mode="precomp", precision="f32_ir", tol_lambda=1e-9)
    x, info = p.solve(bt, 1e-10, 100000)
    assert info.status == B.OK
    assert B.Solver.from_csr(W.small_upwind(32)[0]).layout_info()["rev_bytes"] == 2
