"""Pins of the CPU oracle to what the paper and the mathematics fix (no GPU).

Each test names the passage of arXiv 1904.04093 it checks. None of them compares the oracle
with itself: the references are closed forms printed in the paper, theorems it states,
textbook identities, or library routines (numpy/scipy dense solves).
"""
import numpy as np
import pytest
import scipy.linalg

from conftest import golden
from oracle import gabp as G
from oracle import gabp_loops as GL
from paper_1904_04093_amd import workloads as W


def _graph(a):
    return G.Graph.from_csr(a)


def _dense(a):
    return W.csr_to_dense(a)


def _relerr(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / max(np.linalg.norm(y), 1e-300))


# --------------------------------------------------------------------------------------
# two independent forms of the oracle agree (consistency, not a pin by itself)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_loop_form_matches_vectorized(seed):
    r = W.rng(100, seed)
    a = W.random_walk_summable(30, 0.15, r)          # structurally nonsymmetric
    b = r.uniform(-1, 1, a.n)
    g = _graph(a)
    Lt = np.zeros(g.E)
    m = np.zeros(g.E)
    for s in range(1, 13):
        x, Lt, m, _, _ = G.sweep(g, b, Lt, m)
        xl, Ltl, ml, _ = GL.gabp_loops(a.n, a.rowptr, a.col, a.val, b, s)
        assert _relerr(x, np.array(xl)) < 1e-13
        Ltl_arr = np.array([Ltl[(int(j), int(i))] for i, j in zip(g.dst, g.src)])
        ml_arr = np.array([ml[(int(j), int(i))] for i, j in zip(g.dst, g.src)])
        assert np.allclose(Lt, Ltl_arr, rtol=1e-13, atol=1e-15)
        assert np.allclose(m, ml_arr, rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------------------------------
# Sec. 2.2 facts: GaBP on a tree is Gaussian elimination (exact after diameter updates)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_tree_exact_tridiagonal(seed):
    n = 12
    a = W.random_tridiagonal(n, W.rng(101, seed))
    b = W.rng(102, seed).uniform(-1, 1, n)
    d = _dense(a)
    xs = scipy.linalg.solve(d, b)
    g = _graph(a)
    # the n-th read-off uses n-1 = diameter message updates
    x, _, _ = G.run(g, b, n)
    assert _relerr(x, xs) < 1e-13
    x_early, _, _ = G.run(g, b, n - 1)
    assert _relerr(x_early, xs) > 1e-8
    # on a tree the node precision is the marginal one: Sigma_i = 1 / (A^-1)_ii
    Lt = np.zeros(g.E)
    m = np.zeros(g.E)
    for _ in range(n):
        _, Lt, m, S, _ = G.sweep(g, b, Lt, m)
    S, _ = G.node_totals(g, b, Lt, m)
    assert np.allclose(S, 1.0 / np.diag(np.linalg.inv(d)), rtol=1e-12)


def _tree_diameter(parent):
    n = len(parent)
    adj = [[] for _ in range(n)]
    for v, p in enumerate(parent):
        if p >= 0:
            adj[v].append(p)
            adj[p].append(v)

    def far(s):
        dist = [-1] * n
        dist[s] = 0
        q = [s]
        for u in q:
            for w in adj[u]:
                if dist[w] < 0:
                    dist[w] = dist[u] + 1
                    q.append(w)
        k = int(np.argmax(dist))
        return k, dist[k]

    u, _ = far(0)
    _, d = far(u)
    return d


@pytest.mark.parametrize("seed,one_way", [(0, 0.0), (1, 0.0), (2, 0.3), (3, 0.5)])
def test_tree_exact_random_tree(seed, one_way):
    a, parent = W.random_tree(25, W.rng(103, seed), one_way=one_way)
    b = W.rng(104, seed).uniform(-1, 1, a.n)
    D = _tree_diameter(parent)
    xs = np.linalg.solve(_dense(a), b)
    x, _, _ = G.run(_graph(a), b, D + 1)
    assert _relerr(x, xs) < 1e-13
    if one_way == 0.0:
        x_early, _, _ = G.run(_graph(a), b, D)
        assert _relerr(x_early, xs) > 1e-10


def test_toy_tree_elimination_formulas():
    """The 5x5 example of Sec. 2.1: messages reproduce eqs. elimination_5 and elimination_3.

    The paper's definition of b~_5 in eq. elimination_3 prints A_53 where eliminating x_4
    from row 5 gives A_54; the elimination (and the test) uses A_54.
    """
    r = W.rng(105, 0)
    a = W.toy_5x5(r)
    b = r.uniform(-1, 1, 5)
    A = _dense(a)
    A_ = lambda i, j: A[i - 1, j - 1]
    b_ = lambda i: b[i - 1]
    At33 = A_(3, 3) - A_(3, 1) * A_(1, 3) / A_(1, 1) - A_(3, 2) * A_(2, 3) / A_(2, 2)
    bt3 = b_(3) - A_(3, 1) * b_(1) / A_(1, 1) - A_(3, 2) * b_(2) / A_(2, 2)
    S5 = A_(5, 5) - A_(5, 3) * A_(3, 5) / At33 - A_(5, 4) * A_(4, 5) / A_(4, 4)
    M5 = b_(5) - A_(5, 3) * bt3 / At33 - A_(5, 4) * b_(4) / A_(4, 4)
    At55 = A_(5, 5) - A_(5, 4) * A_(4, 5) / A_(4, 4)
    bt5 = b_(5) - A_(5, 4) * b_(4) / A_(4, 4)
    S3 = At33 - A_(3, 5) * A_(5, 3) / At55
    M3 = bt3 - A_(3, 5) * bt5 / At55
    g = _graph(a)
    Lt = np.zeros(g.E)
    m = np.zeros(g.E)
    for _ in range(4):                     # diameter of the toy tree (1-3-5-4) is 3
        _, Lt, m, _, _ = G.sweep(g, b, Lt, m)
    S, M = G.node_totals(g, b, Lt, m)
    assert S[4] == pytest.approx(S5, rel=1e-14)
    assert M[4] == pytest.approx(M5, rel=1e-13)
    assert S[2] == pytest.approx(S3, rel=1e-14)
    assert M[2] == pytest.approx(M3, rel=1e-13)
    assert M[4] / S[4] == pytest.approx(np.linalg.solve(A, b)[4], rel=1e-13)


# --------------------------------------------------------------------------------------
# Consistency (fixed point = A^-1 b) and convergence (rho(|R~|) < 1, M-matrices)
# --------------------------------------------------------------------------------------

def _rho_abs_R(A):
    D = np.abs(np.diag(A))
    R = np.abs(A) / D[:, None]
    np.fill_diagonal(R, 0.0)
    return float(np.max(np.abs(np.linalg.eigvals(R))))


@pytest.mark.parametrize("seed,sym", [(0, False), (1, False), (2, True), (3, False)])
def test_fixed_point_is_dense_solution(seed, sym):
    r = W.rng(106, seed)
    a = W.random_walk_summable(40, 0.12, r, symmetric_pattern=sym)
    assert _rho_abs_R(_dense(a)) < 1.0              # hypothesis of the convergence theorem
    b = r.uniform(-1, 1, a.n)
    x, info, _, _ = G.solve(_graph(a), b, 1e-15, 5000)
    assert info.status == G.OK
    xs = np.linalg.solve(_dense(a), b)
    assert _relerr(x, xs) < 1e-12
    assert np.abs(_dense(a) @ x - b).max() < 1e-13


def test_fixed_point_upwind_mmatrix():
    a, b = W.small_upwind(32)
    A = _dense(a)
    assert np.all(A[~np.eye(a.n, dtype=bool)] <= 0) and np.all(np.diag(A) > 0)
    assert A[0, 0] == 4.75                            # upwind 32x32 operator, h^2 scaled
    x, info, _, _ = G.solve(_graph(a), b, 1e-13, 20000, check_every=10)
    assert info.status == G.OK
    assert _relerr(x, np.linalg.solve(A, b)) < 1e-10
    assert info.rel_res2 <= 1e-13


def test_paper_7x7_divergence():
    """Sec. 3.4 example: rho(|R~|) ~ 1.03 and point GaBP does not converge (soft pin)."""
    A = np.loadtxt(golden("paper_7x7.txt"), comments="#")
    assert A.shape == (7, 7)
    assert abs(_rho_abs_R(A) - 1.03) < 0.005
    a = W.csr_from_dense(A)
    b = W.rng(107, 0).uniform(-1, 1, 7)
    x, info, _, _ = G.solve(_graph(a), b, 1e-10, 2000)
    assert info.status != G.OK


# --------------------------------------------------------------------------------------
# Sec. 4.1 LFA stencils of one and two parallel sweeps (sweep-count convention)
# --------------------------------------------------------------------------------------

def test_lfa_stencils():
    n = 64
    a = W.laplacian_5pt(n)
    c = 32 * n + 32
    b = np.zeros(a.n)
    b[c] = 1.0
    rows = np.loadtxt(golden("lfa_stencils.txt"), comments="#")
    for sweeps in (1, 2):
        x, _, _ = G.run(_graph(a), b, sweeps)
        expect = np.zeros(a.n)
        for s, ox, oy, v in rows:
            if int(s) == sweeps:
                expect[c + int(ox) + n * int(oy)] = v
        assert np.abs(x - expect).max() < 1e-15


def test_smoother_one_sweep_is_jacobi():
    a, b = W.small_upwind(16)
    g = _graph(a)
    x0 = W.rng(108, 0).uniform(-1, 1, a.n)
    x1 = G.smooth(g, b, x0, 1)
    A = _dense(a)
    assert np.allclose(x1, x0 + (b - A @ x0) / np.diag(A), rtol=1e-14, atol=1e-15)


def test_interior_lambda_closed_form():
    """5-point Laplacian interior: Lt_n = 1/(4 - 3 Lt_{n-1}) from 0: 1/4, 4/13, 13/40, 40/121."""
    n = 64
    a = W.laplacian_5pt(n)
    g = _graph(a)
    c = 32 * n + 32
    into_c = np.nonzero(g.dst == c)[0]
    Lt = np.zeros(g.E)
    m = np.zeros(g.E)
    for expect in (1 / 4, 4 / 13, 13 / 40, 40 / 121):
        _, Lt, m, _, _ = G.sweep(g, np.zeros(a.n), Lt, m)
        assert np.allclose(Lt[into_c], expect, rtol=1e-15)
    # converged: Lt* = 1/3 (stable root), Sigma* = 8/3; first two read-offs 3b/8, (3b+sum)/8
    Lt_s, S_s, _ = G.lambda_phase(g, 1e-15, 200)
    assert S_s[c] == pytest.approx(8 / 3, rel=1e-13)
    b = W.rng(109, 0).uniform(-1, 1, a.n)
    m = np.zeros(g.E)
    x1, m = G.msweep(g, b, Lt_s, S_s, m)
    x2, m = G.msweep(g, b, Lt_s, S_s, m)
    assert x1[c] == pytest.approx(3 * b[c] / 8, rel=1e-13)
    nb = b[c - 1] + b[c + 1] + b[c - n] + b[c + n]
    assert x2[c] == pytest.approx((3 * b[c] + nb) / 8, rel=1e-12)


def test_sequence_interior_closed_form():
    """Per-sweep precision messages from zero (flood): on the Laplacian interior the
    messages of sweeps 1..4 are 1/4, 4/13, 13/40, 40/121 and the read-off precisions are
    4, 3, 36/13, 27/10 (Sigma_s = 4 - 4 Lt_{s-1}); red-black: a red interior node reads
    off with Sigma = 4 and sends 1/4, a black one with 4 - 4/4 = 3 in the same sweep."""
    n = 64
    a = W.laplacian_5pt(n)
    g = _graph(a)
    c = 32 * n + 32
    into_c = np.nonzero(g.dst == c)[0]
    seq = G.lambda_sequence(g, 4)
    for (Lt_s, S_s), lt, sg in zip(seq, (1 / 4, 4 / 13, 13 / 40, 40 / 121),
                                   (4.0, 3.0, 36 / 13, 27 / 10)):
        assert np.allclose(Lt_s[into_c], lt, rtol=1e-15)
        assert S_s[c] == pytest.approx(sg, rel=1e-15)
    col = G.grid_colour(n)
    (Lt1, S1), = G.lambda_sequence(g, 1, col)
    red, black = (c if col[c] == 0 else c + 1), (c if col[c] == 1 else c + 1)
    assert S1[red] == 4.0 and S1[black] == 3.0
    from_red = np.nonzero(g.src == red)[0]
    assert np.allclose(Lt1[from_red], 0.25, rtol=1e-15)


@pytest.mark.parametrize("schedule", ["flood", "redblack", "colour4"])
def test_sequence_smoother_equals_joint_smoother(schedule):
    """Algorithm 3 restarts from zero messages, so the precision messages of its sweeps do
    not depend on the residual: mean-only sweeps with the per-sweep precomputed messages
    reproduce the joint smoother exactly (same operations, same order)."""
    if schedule == "colour4":
        a = W.random_grid_9pt(13, 11, W.rng(121, 0))
        col = G.grid_colour4(13, 11)
    else:
        a, _ = W.small_upwind(16)
        col = G.grid_colour(16) if schedule == "redblack" else None
    g = _graph(a)
    r = W.rng(121, 1)
    b, x0 = r.uniform(-1, 1, a.n), r.uniform(-1, 1, a.n)
    seq = G.lambda_sequence(g, 5, col)
    for mu in (1, 2, 3, 5):
        want = G.smooth(g, b, x0, mu) if col is None else G.smooth_coloured(g, b, x0, mu, col)
        got = G.smooth_seq(g, b, x0, mu, seq, col)
        assert np.array_equal(got, want), (schedule, mu)
    # planted mistake: the converged (frozen) precision messages instead of the sequence
    Lt_s, S_s, _ = G.lambda_phase(g, 1e-14, 2000)
    frozen = G.smooth(g, b, x0, 3, lam=(Lt_s, S_s)) if col is None else \
        G.smooth_coloured(g, b, x0, 3, col, lam=(Lt_s, S_s))
    want = G.smooth(g, b, x0, 3) if col is None else G.smooth_coloured(g, b, x0, 3, col)
    assert _relerr(frozen, want) > 1e-6


# --------------------------------------------------------------------------------------
# Invariances of the rules (algebra on eq. nonsymmetric_GaBP_rules)
# --------------------------------------------------------------------------------------

def _iterates(A, b, sweeps):
    g = _graph(W.csr_from_dense(A))
    out = []
    Lt = np.zeros(g.E)
    m = np.zeros(g.E)
    for _ in range(sweeps):
        x, Lt, m, _, _ = G.sweep(g, b, Lt, m)
        out.append(x)
    return out


def test_invariances():
    r = W.rng(110, 0)
    A = _dense(W.random_walk_summable(25, 0.2, r))
    b = r.uniform(-1, 1, 25)
    b2 = r.uniform(-1, 1, 25)
    D = r.uniform(0.5, 2.0, 25) * np.where(r.random(25) < 0.5, -1, 1)
    P = r.permutation(25)
    base = _iterates(A, b, 8)
    for x0, x1 in zip(base, _iterates(D[:, None] * A, D * b, 8)):      # row scaling
        assert _relerr(x1, x0) < 1e-13
    for x0, x1 in zip(base, _iterates(A * D[None, :], b, 8)):          # column scaling
        assert _relerr(x1, x0 / D) < 1e-13
    for x0, x1 in zip(base, _iterates(-A, -b, 8)):                     # sign flip
        assert _relerr(x1, x0) < 1e-14
    for x0, x1 in zip(base, _iterates(A[np.ix_(P, P)], b[P], 8)):      # permutation
        assert _relerr(x1, x0[P]) < 1e-13
    lin = _iterates(A, b + 2.0 * b2, 8)                                # linearity in b
    for x0, xb, x1 in zip(base, _iterates(A, b2, 8), lin):
        assert _relerr(x1, x0 + 2.0 * xb) < 1e-13


def test_triangular_is_back_substitution():
    r = W.rng(111, 0)
    n = 10
    L = np.tril(r.uniform(-1, 1, (n, n)), -1) + np.diag(r.uniform(1.0, 2.0, n))
    b = r.uniform(-1, 1, n)
    xs = scipy.linalg.solve_triangular(L, b, lower=True)
    xn = _iterates(L, b, n)
    assert _relerr(xn[-1], xs) < 1e-13            # longest path n-1 updates
    assert _relerr(xn[-2], xs) > 1e-10


def test_symmetric_matches_conventional_rules():
    r = W.rng(112, 0)
    n = 20
    M = np.where(r.random((n, n)) < 0.2, r.uniform(-1, 1, (n, n)), 0.0)
    A = np.triu(M, 1)
    A = A + A.T
    np.fill_diagonal(A, 1.4 * np.abs(A).sum(1) + 0.1)
    b = r.uniform(-1, 1, n)
    a = W.csr_from_dense(A)
    xs = _iterates(A, b, 10)
    for s in range(1, 11):
        xc = GL.conventional_gabp_loops(n, a.rowptr, a.col, a.val, b, s)
        assert _relerr(xs[s - 1], np.array(xc)) < 1e-12


# --------------------------------------------------------------------------------------
# Precomputed Lambda~ and the FP32-message refinement reach the same fixed point
# --------------------------------------------------------------------------------------

def test_precomp_reaches_dense_solution():
    a, b = W.small_upwind(32)
    g = _graph(a)
    x, info = G.solve_precomp(g, b, 1e-13, 20000, check_every=10)
    assert info.status == G.OK
    assert _relerr(x, np.linalg.solve(_dense(a), b)) < 1e-10


def test_ir_fp32_messages_reaches_fp64_accuracy():
    """Refinement's fixed point is A^-1 b however inexact the FP32 inner solves are: the
    converged x equals the dense solution far below FP32 resolution."""
    a, b = W.small_upwind(32)
    g = _graph(a)
    Lt, S, _ = G.lambda_phase(g, 1e-7, 1000)
    x, info = G.ir_solve(g, b, 1e-12, (Lt.astype(np.float32), (1.0 / S).astype(np.float32)))
    assert info.status == G.OK
    assert info.outer_iters >= 2          # one FP32 inner solve alone cannot get there
    assert _relerr(x, np.linalg.solve(_dense(a), b)) < 1e-9


def test_ir_on_a_tree_needs_one_exact_inner_solve_per_step():
    """On a tridiagonal matrix GaBP is exact after diameter updates (tree exactness, Sec.
    2.3), so each inner solve of n + 1 sweeps is exact up to FP32 rounding: every outer step
    must cut the residual by about the FP32 unit roundoff times the condition number."""
    a = W.random_tridiagonal(24, W.rng(120, 0))
    g = _graph(a)
    b = W.rng(120, 1).uniform(-1, 1, a.n)
    Lt, S, _ = G.lambda_phase(g, 0.0, a.n)
    lam32 = (Lt.astype(np.float32), (1.0 / S).astype(np.float32))
    x, info = G.ir_solve(g, b, 1e-14, lam32, check_every=a.n + 1, inner_tol=0.0,
                         max_inner=a.n + 1)
    A = _dense(a)
    assert info.status == G.OK
    assert info.outer_iters <= 4
    assert _relerr(x, np.linalg.solve(A, b)) < 1e-13


def test_ir_planted_mistake_fails():
    """A wrong sign in the outer residual (b + A x) breaks convergence to the dense
    solution: the pin above sees it."""
    a, b = W.small_upwind(16)
    g = _graph(a)
    Lt, S, _ = G.lambda_phase(g, 1e-7, 1000)
    lam32 = (Lt.astype(np.float32), (1.0 / S).astype(np.float32))
    xs = np.linalg.solve(_dense(a), b)

    class WrongSign(G.Graph):
        def residual(self, bb, xx):        # planted: refinement sees b + A x
            return bb + self.matvec(xx)
    bad = WrongSign.from_csr(a)
    x, info = G.ir_solve(bad, b, 1e-12, lam32, max_sweeps=20000)
    assert not (info.status == G.OK and _relerr(x, xs) < 1e-9)


# --------------------------------------------------------------------------------------
# Red-black schedule (the paper's red-black GaBP)
# --------------------------------------------------------------------------------------

def test_redblack_first_sweep_closed_form():
    """Sweep 1 from zero messages: red nodes read D^-1 b; black nodes see one elimination
    of their red neighbours: x_j = (b_j - sum_k A_jk b_k / A_kk) / (A_jj - sum_k A_jk A_kj / A_kk).
    """
    a, b = W.small_upwind(8)
    g = _graph(a)
    colour = G.grid_colour(8)
    x, _, _ = G.sweep_coloured(g, b, np.zeros(g.E), np.zeros(g.E), colour)
    A = _dense(a)
    for j in range(a.n):
        if colour[j] == 0:
            assert x[j] == pytest.approx(b[j] / A[j, j], rel=1e-15)
        else:
            ks = [k for k in range(a.n) if k != j and A[j, k] != 0]
            num = b[j] - sum(A[j, k] * b[k] / A[k, k] for k in ks)
            den = A[j, j] - sum(A[j, k] * A[k, j] / A[k, k] for k in ks)
            assert x[j] == pytest.approx(num / den, rel=1e-13)


@pytest.mark.parametrize("precomp", [False, True])
def test_redblack_fixed_point_is_dense_solution(precomp):
    a, b = W.small_upwind(16)
    g = _graph(a)
    colour = G.grid_colour(16)
    lam = None
    if precomp:
        Lt, S, _ = G.lambda_phase(g, 1e-15, 500)
        lam = (Lt, S)
    Lt = np.zeros(g.E) if lam is None else lam[0]
    m = np.zeros(g.E)
    for _ in range(400):
        x, Lt, m = G.sweep_coloured(g, b, Lt, m, colour, lambda_fixed=lam)
    assert _relerr(x, np.linalg.solve(_dense(a), b)) < 1e-12


def test_four_colour_schedule_first_class_reads_jacobi_and_fixed_point():
    # 4-colour GaBP (Sec. 5, mixed-derivative problem) on a 9-point stencil: the first colour
    # class reads off from zero messages (a Jacobi step); the fixed point is A^-1 b
    n = 15
    a, b, _ = W.sec5_problem("mixed_derivative", n, eps=0.01)
    A = _dense(a)
    colour = G.grid_colour4(n)
    g = _graph(a)
    # proper for the 9-point stencil: no stored coupling inside a colour class
    assert not np.any(colour[g.dst] == colour[g.src])
    x, Lt, m = G.sweep_coloured(g, b, np.zeros(g.E), np.zeros(g.E), colour)
    first = colour == 0
    assert np.allclose(x[first], b[first] / np.diag(A)[first], rtol=1e-15, atol=0)
    # fixed point on a dominant 9-point operator (the mixed-derivative one is nearly
    # non-elliptic and GaBP alone does not converge on it)
    r = W.rng(120, 0)
    D = np.zeros((n * n, n * n))
    for i in range(n * n):
        iy, ix = divmod(i, n)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                jx, jy = ix + dx, iy + dy
                if (dx or dy) and 0 <= jx < n and 0 <= jy < n:
                    D[i, jy * n + jx] = -r.uniform(0.2, 1.0)
        D[i, i] = 1.2 * np.abs(D[i]).sum()
    g = _graph(W.csr_from_dense(D))
    x, Lt, m = G.sweep_coloured(g, b, np.zeros(g.E), np.zeros(g.E), colour)
    for _ in range(400):
        x, Lt, m = G.sweep_coloured(g, b, Lt, m, colour)
    assert _relerr(x, np.linalg.solve(D, b)) < 1e-10


# --------------------------------------------------------------------------------------
# The pins catch plausible mistakes: each mutation of the sweep below breaks some pin
# (planted in a copy of the oracle's sweep on the CPU; the oracle itself is untouched)
# --------------------------------------------------------------------------------------

def _mutated_sweep(kind):
    def sweep(g, b, Lt, m, lambda_fixed=False):
        S, M = G.node_totals(g, b, Lt, m)
        if kind == "aji_in_sigma":          # transposed operand in the precision sum
            S = g.diag + np.bincount(g.dst, weights=Lt * g.a_ij, minlength=g.n)
        x = M / S
        back_L = G._gather(Lt, g.rev)
        back_m = G._gather(m, g.rev)
        if kind == "no_cavity":             # dropped term: reverse message not excluded
            back_L = 0 * back_L
            back_m = 0 * back_m
        a = g.a_ji if kind == "aji_numerator" else g.a_ij
        Lt_new = -a / (S[g.src] - back_L * g.a_ij)
        if kind == "sign":                  # wrong sign
            Lt_new = -Lt_new
        m_new = Lt_new * (M[g.src] - back_m)
        if kind == "receiver_total":        # wrong index: receiver's totals instead of sender's
            m_new = Lt_new * (M[g.dst] - back_m)
        return x, Lt_new, m_new, S, M
    return sweep


@pytest.mark.parametrize("kind", ["aji_in_sigma", "no_cavity", "aji_numerator", "sign",
                                  "receiver_total"])
def test_pins_detect_planted_mistakes(kind, monkeypatch):
    monkeypatch.setattr(G, "sweep", _mutated_sweep(kind))
    failures = 0
    # pin 1: tree exactness (nonsymmetric tridiagonal)
    a = W.random_tridiagonal(12, W.rng(101, 0))
    b = W.rng(102, 0).uniform(-1, 1, 12)
    with np.errstate(all="ignore"):
        x, _, _ = G.run(_graph(a), b, 12)
    failures += not (_relerr(x, np.linalg.solve(_dense(a), b)) < 1e-13)
    # pin 2: LFA two-sweep stencil
    n = 16
    lap = W.laplacian_5pt(n)
    bb = np.zeros(lap.n)
    bb[8 * n + 8] = 1.0
    with np.errstate(all="ignore"):
        x2, _, _ = G.run(_graph(lap), bb, 2)
    failures += not (abs(x2[8 * n + 8] - 1 / 3) < 1e-15 and abs(x2[8 * n + 9] - 1 / 12) < 1e-15)
    assert failures >= 1, f"planted mistake {kind} passed every pin"


# The coloured and the mean-only sweeps get the same treatment: each plausible mistake,
# planted in a copy on the CPU, breaks one of the pins above that do not go through the
# flood sweep (red-black first-sweep closed form, coloured and mean-only fixed points,
# the interior read-offs 3b/8 and (3b + sum)/8 of Sec. 4.2's precomputed form).

def _mutated_coloured(kind):
    def sweep_coloured(g, b, Lt, m, colour, lambda_fixed=None):
        colour = np.asarray(colour)
        x = np.zeros(g.n)
        Lt, m = Lt.copy(), m.copy()
        S0, M0 = G.node_totals(g, b, Lt, m)
        for c in range(int(colour.max()) + 1):
            if kind == "stale_totals":          # Jacobi: totals from the start of the sweep
                S, M = S0, M0
            else:
                S, M = G.node_totals(g, b, Lt, m)
            if lambda_fixed is not None:
                S = lambda_fixed[1]
            sel = colour == c
            x[sel] = M[sel] / S[sel]
            upd = (colour[g.dst] if kind == "receiver_class" else colour[g.src]) == c
            back_m = G._gather(m, g.rev)
            if kind == "no_cavity":
                back_m = 0 * back_m
            if lambda_fixed is None:
                with np.errstate(all="ignore"):
                    L_new = -g.a_ij / (S[g.src] - G._gather(Lt, g.rev) * g.a_ij)
                Lt = np.where(upd, L_new, Lt)
            else:
                L_new = lambda_fixed[0]
            m = np.where(upd, L_new * (M[g.src] - back_m), m)
        return x, Lt, m
    return sweep_coloured


@pytest.mark.parametrize("kind", ["stale_totals", "receiver_class", "no_cavity"])
def test_coloured_pins_detect_planted_mistakes(kind, monkeypatch):
    monkeypatch.setattr(G, "sweep_coloured", _mutated_coloured(kind))
    checks = [test_redblack_first_sweep_closed_form,
              lambda: test_redblack_fixed_point_is_dense_solution(False),
              lambda: test_redblack_fixed_point_is_dense_solution(True)]
    failures = 0
    for check in checks:
        try:
            with np.errstate(all="ignore"):
                check()
        except AssertionError:
            failures += 1
    assert failures >= 1, f"planted mistake {kind} passed every coloured-sweep pin"


def _mutated_msweep(kind):
    def msweep(g, b, Lt_star, S_star, m):
        M = b + np.bincount(g.dst, weights=m, minlength=g.n)
        if kind == "receiver_total":            # receiver's total instead of the sender's
            back = G._gather(m, g.rev)
            return M / S_star, Lt_star * (M[g.dst] - back)
        if kind == "no_cavity":
            return M / S_star, Lt_star * M[g.src]
        if kind == "stale_readoff":             # read-off before the incoming sum
            return b / S_star, Lt_star * (M[g.src] - G._gather(m, g.rev))
        return M / S_star, Lt_star * (M[g.src] - G._gather(m, g.rev))
    return msweep


@pytest.mark.parametrize("kind", ["receiver_total", "no_cavity", "stale_readoff"])
def test_mean_only_pins_detect_planted_mistakes(kind, monkeypatch):
    monkeypatch.setattr(G, "msweep", _mutated_msweep(kind))
    failures = 0
    for check in (test_interior_lambda_closed_form, test_precomp_reaches_dense_solution):
        try:
            with np.errstate(all="ignore"):
                check()
        except AssertionError:
            failures += 1
    assert failures >= 1, f"planted mistake {kind} passed every mean-only pin"


# The precision-message precomputes: planted mistakes in copies of lambda_phase (converged
# Lt*) and lambda_sequence (the per-sweep Lt of the smoother) each break a pin above.

def _mutated_lambda_phase(kind):
    def lambda_phase(g, tol_lambda=1e-14, max_sweeps=10000):
        Lt = np.zeros(g.E)
        zeros = np.zeros(g.n)
        a_num = g.a_ji if kind == "transposed" else g.a_ij
        for _ in range(max_sweeps):
            S, _ = G.node_totals(g, zeros, Lt, np.zeros(g.E))
            back = 0 * Lt if kind == "no_cavity" else G._gather(Lt, g.rev)
            with np.errstate(all="ignore"):
                Lt_new = -a_num / (S[g.src] - back * g.a_ij)
            done = float(np.abs(Lt_new - Lt).max()) <= tol_lambda * float(np.abs(Lt_new).max())
            Lt = Lt_new
            if tol_lambda > 0 and done:
                break
        S_star, _ = G.node_totals(g, zeros, Lt, np.zeros(g.E))
        if kind == "diag_only":                 # Sigma* without the incoming precisions
            S_star = g.diag.copy()
        return Lt, S_star, max_sweeps
    return lambda_phase


@pytest.mark.parametrize("kind", ["transposed", "no_cavity", "diag_only"])
def test_lambda_phase_pins_detect_planted_mistakes(kind, monkeypatch):
    monkeypatch.setattr(G, "lambda_phase", _mutated_lambda_phase(kind))
    failures = 0
    for check in (test_interior_lambda_closed_form, test_precomp_reaches_dense_solution):
        try:
            with np.errstate(all="ignore"):
                check()
        except AssertionError:
            failures += 1
    assert failures >= 1, f"planted mistake {kind} passed every precompute pin"


def _mutated_lambda_sequence(kind):
    real = G.lambda_sequence

    def lambda_sequence(g, depth, colour=None):
        if kind == "shifted":                   # read-off precisions one sweep late
            seq = real(g, depth + 1, colour)
            return [(seq[s][0], seq[s + 1][1]) for s in range(depth)]
        if kind == "all_classes":               # a coloured sweep updating every class at once
            return real(g, depth, None)
        if kind == "transposed":
            gt = g.transposed()
            return [(Lt, S) for Lt, S in real(gt, depth, colour)]
        raise AssertionError(kind)
    return lambda_sequence


@pytest.mark.parametrize("kind", ["shifted", "all_classes", "transposed"])
def test_lambda_sequence_pins_detect_planted_mistakes(kind, monkeypatch):
    monkeypatch.setattr(G, "lambda_sequence", _mutated_lambda_sequence(kind))
    failures = 0
    for check in (test_sequence_interior_closed_form,
                  lambda: test_sequence_smoother_equals_joint_smoother("flood"),
                  lambda: test_sequence_smoother_equals_joint_smoother("redblack")):
        try:
            with np.errstate(all="ignore"):
                check()
        except AssertionError:
            failures += 1
    assert failures >= 1, f"planted mistake {kind} passed every sequence pin"


def test_unplanted_copies_pass_every_pin(monkeypatch):
    """The copies the planted mistakes go into are faithful: with nothing planted they pass
    every pin they are run against, so each failure above comes from its mistake."""
    monkeypatch.setattr(G, "sweep", _mutated_sweep("none"))
    a = W.random_tridiagonal(12, W.rng(101, 0))
    b = W.rng(102, 0).uniform(-1, 1, 12)
    x, _, _ = G.run(_graph(a), b, 12)
    assert _relerr(x, np.linalg.solve(_dense(a), b)) < 1e-13
    test_lfa_stencils()
    monkeypatch.setattr(G, "sweep_coloured", _mutated_coloured("none"))
    test_redblack_first_sweep_closed_form()
    test_redblack_fixed_point_is_dense_solution(False)
    test_redblack_fixed_point_is_dense_solution(True)
    monkeypatch.setattr(G, "msweep", _mutated_msweep("none"))
    monkeypatch.setattr(G, "lambda_phase", _mutated_lambda_phase("none"))
    test_interior_lambda_closed_form()
    test_precomp_reaches_dense_solution()
