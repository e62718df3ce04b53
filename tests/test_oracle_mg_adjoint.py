"""Pins of the multigrid and adjoint oracles (no GPU).

Multigrid: the transfer operators of Sec. 4 (full weighting, bilinear interpolation) against
their textbook identities, and the V-cycle against the textbook contraction of red-black
Gauss-Seidel on the Poisson problem. Adjoint: central finite differences and dense-LU
solves (library routines), plus the identity g^T x = lambda^T b.
"""
import numpy as np
import pytest

from oracle import adjoint as AD
from oracle import gabp as G
from oracle import mg as MG
from paper_1904_04093_amd import workloads as W


def _unit_images(fn, n_in, n_out):
    M = np.zeros((n_out, n_in))
    for k in range(n_in):
        e = np.zeros(n_in)
        e[k] = 1.0
        M[:, k] = fn(e)
    return M


def test_full_weighting_is_quarter_transpose_of_bilinear():
    n_c = 7
    n_f = 2 * n_c + 1
    P = _unit_images(lambda e: MG.prolong_bilinear(e, n_c), n_c * n_c, n_f * n_f)
    R = _unit_images(lambda e: MG.restrict_fw(e, n_f), n_f * n_f, n_c * n_c)
    assert np.array_equal(R, P.T / 4.0)
    assert np.allclose(R.sum(1)[(n_c + 1) // 2], 1.0)     # weights sum to one inside


def test_bilinear_reproduces_bilinear_functions():
    n_c = 7
    n_f = 2 * n_c + 1
    f = lambda x, y: (0.3 + 1.7 * x) * (-0.2 + 0.9 * y)
    hc, hf = 1.0 / (n_c + 1), 1.0 / (n_f + 1)
    t = (np.arange(n_c) + 1) * hc
    yc, xc = np.meshgrid(t, t, indexing="ij")
    e = MG.prolong_bilinear(f(xc, yc).reshape(-1), n_c).reshape(n_f, n_f)
    t = (np.arange(n_f) + 1) * hf
    yf, xf = np.meshgrid(t, t, indexing="ij")
    inner = (slice(1, n_f - 1), slice(1, n_f - 1))    # stencils that avoid the boundary
    assert np.abs(e[inner] - f(xf, yf)[inner]).max() < 1e-15


def test_full_weighting_of_linear_function():
    n_f = 15
    hf = 1.0 / (n_f + 1)
    t = (np.arange(n_f) + 1) * hf
    yf, xf = np.meshgrid(t, t, indexing="ij")
    r = (2.0 + 3.0 * xf - 1.0 * yf).reshape(-1)
    rc = MG.restrict_fw(r, n_f).reshape(7, 7)
    tc = (np.arange(7) + 1) * (2 * hf)
    yc, xc = np.meshgrid(tc, tc, indexing="ij")
    assert np.abs(rc - (2.0 + 3.0 * xc - 1.0 * yc)).max() < 1e-14


def test_vcycle_rbgs_poisson_textbook_contraction():
    levels = W.mg_hierarchy(6, coarsest=3, kx=1.0, ky=1.0, peclet=0.0)
    h = MG.Hierarchy(levels, smoother="rbgs", nu1=2, nu2=2)
    b = W.rng(120, 0).uniform(-1, 1, levels[0].n)
    x, hist = h.solve(b, 1e-10, 20)
    rates = np.array(hist[1:]) / np.array(hist[:-1])
    assert rates[2:].max() < 0.15
    assert hist[-1] <= 1e-10


def test_vcycle_exact_coarse_solve_two_levels():
    """Two levels with no smoothing: x = P A_c^{-1} R b exactly (dense check)."""
    levels = W.mg_hierarchy(3, coarsest=3, kx=1.0, ky=1.0, peclet=1.0)
    assert [a.n for a in levels] == [49, 9]
    h = MG.Hierarchy(levels, smoother="rbgs", nu1=0, nu2=0)
    b = W.rng(121, 0).uniform(-1, 1, 49)
    x = h.vcycle(b, np.zeros(49))
    Ac = W.csr_to_dense(levels[1])
    P = _unit_images(lambda e: MG.prolong_bilinear(e, 3), 9, 49)
    assert np.allclose(x, P @ np.linalg.solve(Ac, P.T @ b / 4.0), rtol=1e-13, atol=1e-15)


def _theta_setup(n=16, t=0):
    theta = W.theta_problem(n, t)
    b = W.rng(5, 101).uniform(-1, 1, n * n)
    xt = W.rng(5, 100).uniform(-1, 1, n * n)
    return theta, b, xt


def _loss(n, theta, b, xt):
    A = W.csr_to_dense(W.theta_operator(n, theta))
    x = np.linalg.solve(A, b)
    return 0.5 * float((x - xt) @ (x - xt))


def test_adjoint_gradient_matches_central_differences():
    n = 16
    theta, b, xt = _theta_setup(n)
    a, jptr, jnnz, jw = W.theta_jacobian(n, theta)
    ref = AD.dense_reference(W.csr_to_dense(a), b, xt, a.row_of_nnz(), a.col,
                             jac=(jptr, jnnz, jw))
    eps = 1e-6
    ps = W.rng(122, 0).choice(n * n, 16, replace=False)
    fd = []
    for p in ps:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += eps
        tm[p] -= eps
        fd.append((_loss(n, tp, b, xt) - _loss(n, tm, b, xt)) / (2 * eps))
    fd = np.array(fd)
    # norm-wise over the sampled parameters: the FD round-off floor (~eps_mach L / eps)
    # dominates tiny individual components
    assert np.linalg.norm(fd - ref["dtheta"][ps]) <= 1e-6 * np.linalg.norm(fd)


def test_adjoint_dot_product_identity_and_gabp_adjoint():
    n = 16
    theta, b, xt = _theta_setup(n, 1)
    a, jptr, jnnz, jw = W.theta_jacobian(n, theta)
    ref = AD.dense_reference(W.csr_to_dense(a), b, xt, a.row_of_nnz(), a.col,
                             jac=(jptr, jnnz, jw))
    gx = ref["x"] - xt
    assert float(gx @ ref["x"]) == pytest.approx(float(ref["lam"] @ b), rel=1e-12)
    out = AD.gabp_adjoint(G.Graph.from_csr(a), b, xt, 1e-14, 20000, jac=(jptr, jnnz, jw),
                          check_every=10)
    assert np.linalg.norm(out["lam"] - ref["lam"]) <= 1e-9 * np.linalg.norm(ref["lam"])
    assert np.linalg.norm(out["dtheta"] - ref["dtheta"]) <= 1e-8 * np.linalg.norm(ref["dtheta"])


def test_transposed_graph_swaps_coefficients():
    r = W.rng(123, 0)
    a = W.random_walk_summable(20, 0.2, r)
    g = G.Graph.from_csr(a)
    gt = g.transposed()
    assert np.array_equal(gt.dense(), g.dense().T)
    b = r.uniform(-1, 1, 20)
    x, info, _, _ = G.solve(gt, b, 1e-14, 5000)
    assert np.allclose(x, np.linalg.solve(g.dense().T, b), rtol=1e-11)


# The multigrid pins catch plausible mistakes: each one below, planted in a copy on the CPU
# (the oracle itself untouched), breaks at least one of the transfer-operator identities or
# the textbook V-cycle checks above.

def _restrict_no_corners(r, n_f):
    n_c = (n_f - 1) // 2
    R = np.asarray(r, dtype=np.float64).reshape(n_f, n_f)
    c = 4.0 * R[1::2, 1::2]
    c += 2.0 * (R[0:-1:2, 1::2] + R[2::2, 1::2] + R[1::2, 0:-1:2] + R[1::2, 2::2])
    return (c / 16.0).reshape(-1)


def _prolong_constant_in_y(e_c, n_c):
    n_f = 2 * n_c + 1
    E = np.zeros((n_c + 2, n_c + 2))
    E[1:-1, 1:-1] = np.asarray(e_c, dtype=np.float64).reshape(n_c, n_c)
    F = np.zeros((n_f + 2, n_f + 2))
    F[::2, ::2] = E
    F[::2, 1::2] = 0.5 * (E[:, :-1] + E[:, 1:])
    F[1::2, :] = F[0:-1:2, :]                   # no average between coarse rows
    return F[1:-1, 1:-1].reshape(-1)


def _rbgs_jacobi(g, b, x, n, sweeps):
    x = np.array(x, dtype=np.float64)
    off = g.rows != g.cols
    for _ in range(sweeps):
        s = np.bincount(g.rows[off], weights=g.vals[off] * x[g.cols[off]], minlength=g.n)
        x = (b - s) / g.diag                    # both colours from the old iterate
    return x


def _vcycle_mutant(kind):
    def vcycle(self, b, x, l=0):
        g = self.graphs[l]
        if l == len(self.graphs) - 1:
            return self.coarse @ b
        x = self._smooth(l, b, x, self.nu1)
        r = b if kind == "restrict_b" else g.residual(b, x)
        ec = self.vcycle(MG.restrict_fw(r, self.sides[l]),
                         np.zeros(self.graphs[l + 1].n), l + 1)
        e = MG.prolong_bilinear(ec, self.sides[l + 1])
        x = x - e if kind == "sign" else x + e
        return self._smooth(l, b, x, self.nu2)
    return vcycle


@pytest.mark.parametrize("kind", ["restrict_no_corners", "prolong_constant_in_y",
                                  "rbgs_jacobi", "sign", "restrict_b"])
def test_mg_pins_detect_planted_mistakes(kind, monkeypatch):
    if kind == "restrict_no_corners":
        monkeypatch.setattr(MG, "restrict_fw", _restrict_no_corners)
    elif kind == "prolong_constant_in_y":
        monkeypatch.setattr(MG, "prolong_bilinear", _prolong_constant_in_y)
    elif kind == "rbgs_jacobi":
        monkeypatch.setattr(MG, "rbgs", _rbgs_jacobi)
    else:
        monkeypatch.setattr(MG.Hierarchy, "vcycle", _vcycle_mutant(kind))
    failures = 0
    for check in (test_full_weighting_is_quarter_transpose_of_bilinear,
                  test_bilinear_reproduces_bilinear_functions,
                  test_full_weighting_of_linear_function,
                  test_vcycle_rbgs_poisson_textbook_contraction,
                  test_vcycle_exact_coarse_solve_two_levels):
        try:
            with np.errstate(all="ignore"):
                check()
        except AssertionError:
            failures += 1
    assert failures >= 1, f"planted mistake {kind} passed every multigrid pin"


def test_entry_gradient_matches_central_differences():
    """dL/dA_e = -lambda_i x_j for the stored entry e = (i, j), checked entry by entry
    against central differences of L(A^-1 b) on a nonsymmetric upwind matrix (A_ij != A_ji,
    so a transposed gradient cannot pass, unlike the theta chain, whose weights are equal
    for A_ij and A_ji)."""
    a, _ = W.small_upwind(6)
    A = W.csr_to_dense(a)
    r = W.rng(124, 0)
    b = r.uniform(-1, 1, a.n)                    # O(1) x and gradient: FD floor far below
    xt = 0.5 * np.linalg.solve(A, b) + r.uniform(-0.1, 0.1, a.n)
    rows, cols = a.row_of_nnz(), a.col
    ref = AD.dense_reference(A, b, xt, rows, cols)
    loss = lambda M: 0.5 * float(((x := np.linalg.solve(M, b)) - xt) @ (x - xt))
    eps = 1e-6
    es = W.rng(124, 1).choice(a.nnz, 24, replace=False)
    fd = []
    for e in es:
        Ap, Am = A.copy(), A.copy()
        Ap[rows[e], cols[e]] += eps
        Am[rows[e], cols[e]] -= eps
        fd.append((loss(Ap) - loss(Am)) / (2 * eps))
    fd = np.array(fd)
    assert np.linalg.norm(fd - ref["G"][es]) <= 1e-6 * np.linalg.norm(fd)


# The adjoint pins catch plausible mistakes as well (planted in copies, on the CPU): a
# transposed or sign-flipped entry gradient, dropped Jacobian weights, and an adjoint solve
# with A in place of A^T each break a finite-difference or dense-LU check above.

def _adjoint_mutant(kind, monkeypatch):
    if kind == "gradient_transposed":
        monkeypatch.setattr(AD, "nnz_gradient",
                            lambda rows, cols, lam, x: -np.asarray(lam)[cols] * np.asarray(x)[rows])
    elif kind == "gradient_sign":
        monkeypatch.setattr(AD, "nnz_gradient",
                            lambda rows, cols, lam, x: np.asarray(lam)[rows] * np.asarray(x)[cols])
    elif kind == "unweighted_chain":
        real = AD.reduce_to_params
        monkeypatch.setattr(AD, "reduce_to_params",
                            lambda G_, jptr, jnnz, jw: real(G_, jptr, jnnz, np.ones(len(jw))))
    elif kind == "forward_operator":
        monkeypatch.setattr(G.Graph, "transposed", lambda self: self)


@pytest.mark.parametrize("kind", ["gradient_transposed", "gradient_sign", "unweighted_chain",
                                  "forward_operator"])
def test_adjoint_pins_detect_planted_mistakes(kind, monkeypatch):
    _adjoint_mutant(kind, monkeypatch)
    failures = 0
    for check in (test_adjoint_gradient_matches_central_differences,
                  test_entry_gradient_matches_central_differences,
                  test_adjoint_dot_product_identity_and_gabp_adjoint):
        try:
            check()
        except AssertionError:
            failures += 1
    assert failures >= 1, f"planted mistake {kind} passed every adjoint pin"


def test_unplanted_vcycle_copy_passes_every_pin(monkeypatch):
    """The V-cycle copy the planted mistakes go into passes the V-cycle pins unchanged."""
    monkeypatch.setattr(MG.Hierarchy, "vcycle", _vcycle_mutant("none"))
    test_vcycle_rbgs_poisson_textbook_contraction()
    test_vcycle_exact_coarse_solve_two_levels()
