"""Vectorized FP64 oracle for flood GaBP on nonsymmetric systems (test infrastructure only).

Same iteration as ``oracle.gabp_loops`` written with numpy edge arrays so that it reaches
grids of a few million unknowns. Paper references (arXiv 1904.04093):

* graph: edge j -> i iff A_ij != 0 (Sec. 2.3, construction of the directed graph);
* messages (Lt_ji, m_ji) = (Lambda_ji / A_ji, mu_ji Lambda_ji) (eq. nonsymmetric_GaBP_messages);
* update and read-off rules: eq. nonsymmetric_GaBP_rules; Algorithm 1;
* flood ("parallel") schedule: Sec. 2.2, remark after eq. GaBP_rules, and Sec. 2.3;
* stopping rule: a norm of b - A x (Algorithm 1; Sec. 5 uses the max norm);
* Lt does not depend on b and can be computed once and reused (Sec. 2.3, remark after the
  stopping criteria; Sec. 4.2);
* error-correction smoother (Algorithm 3).

Readings of points the paper leaves open (each listed in the design notes):

* initial messages are zero;
* one *sweep* = one iteration of Algorithm 1: read off x from the current messages, then
  update every message; so the s-th read-off uses s-1 message updates (pinned by the LFA
  stencils of Sec. 4.1);
* the residual test runs on the read-off of the sweep just done, every ``check_every``
  sweeps and at ``max_sweeps``;
* stop when ||b - A x||_2 / ||b||_2 <= tol (the max norm is reported as well);
* a zero or non-finite cavity precision is a numeric failure (no damping, no pivoting);
* Lt counts as converged when max|dLt| <= tol_lambda * max|Lt| between consecutive updates.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

OK, MAXSWEEPS, ENUMERIC = 0, 1, -4


class Graph:
    """Directed message graph of a square CSR matrix (oracle's own construction).

    Edge arrays are ordered by receiver, then sender (the CSR order of the off-diagonal
    nonzeros). For edge e = (src j -> dst i): ``a_ij[e] = A_ij`` (CSR value at row i, col j),
    ``a_ji[e] = A_ji`` (0 if absent), ``rev[e]`` = edge i -> j or -1.
    """

    def __init__(self, n, rowptr, col, val):
        rowptr = np.asarray(rowptr, dtype=np.int64)
        col = np.asarray(col, dtype=np.int64)
        val = np.asarray(val, dtype=np.float64)
        self.n = int(n)
        rows = np.repeat(np.arange(self.n), np.diff(rowptr))
        self.rows, self.cols, self.vals = rows, col, val
        on_diag = rows == col
        self.diag = np.zeros(self.n)
        self.diag[rows[on_diag]] = val[on_diag]
        keep = (~on_diag) & (val != 0.0)
        self.dst = rows[keep]
        self.src = col[keep]
        self.a_ij = val[keep]
        # rev: position of the edge i -> j (CSR entry (j, i) with A_ji != 0), else -1
        key = self.dst * self.n + self.src
        rkey = self.src * self.n + self.dst
        order = np.argsort(key, kind="stable")
        skey = key[order]
        self.rev = np.full(len(key), -1, dtype=np.int64)
        if len(key):
            loc = np.minimum(np.searchsorted(skey, rkey), len(key) - 1)
            found = skey[loc] == rkey
            self.rev[found] = order[loc[found]]
        self.a_ji = np.where(self.rev >= 0, self.a_ij[np.maximum(self.rev, 0)], 0.0)
        self.E = len(self.dst)

    @classmethod
    def from_csr(cls, a):
        return cls(a.n, a.rowptr, a.col, a.val)

    def transposed(self):
        """Graph of A^T (same nonzeros, rows and columns swapped)."""
        order = np.lexsort((self.rows, self.cols))
        rows_t, cols_t, vals_t = self.cols[order], self.rows[order], self.vals[order]
        rowptr = np.zeros(self.n + 1, dtype=np.int64)
        np.add.at(rowptr, rows_t + 1, 1)
        return Graph(self.n, np.cumsum(rowptr), cols_t, vals_t)

    def matvec(self, x):
        y = np.bincount(self.rows, weights=self.vals * x[self.cols], minlength=self.n)
        return y

    def residual(self, b, x):
        return b - self.matvec(x)

    def dense(self):
        d = np.zeros((self.n, self.n))
        d[self.rows, self.cols] = self.vals
        return d


def _gather(arr, rev):
    return np.where(rev >= 0, arr[np.maximum(rev, 0)], 0.0)


def node_totals(g: Graph, b, Lt, m):
    """Sigma_j = A_jj + sum_k Lt_kj A_kj and m_j = b_j + sum_k m_kj (Algorithm 1)."""
    S = g.diag + np.bincount(g.dst, weights=Lt * g.a_ji, minlength=g.n)
    M = b + np.bincount(g.dst, weights=m, minlength=g.n)
    return S, M


def sweep(g: Graph, b, Lt, m, lambda_fixed=False):
    """One flood iteration. Returns (x, Lt_new, m_new, Sigma, M).

    x is the read-off from the incoming messages (Lt, m). For edge j -> i the new message is
    Lt_ji = -A_ij / (Sigma_j - Lt_ij A_ij), m_ji = Lt_ji (M_j - m_ij); with
    ``lambda_fixed`` Lt is kept as given (precomputed Lambda~, Sec. 4.2).
    """
    S, M = node_totals(g, b, Lt, m)
    x = M / S
    back_L = _gather(Lt, g.rev)
    back_m = _gather(m, g.rev)
    if lambda_fixed:
        Lt_new = Lt
    else:
        with np.errstate(divide="ignore", invalid="ignore"):
            Lt_new = -g.a_ij / (S[g.src] - back_L * g.a_ij)
    m_new = Lt_new * (M[g.src] - back_m)
    return x, Lt_new, m_new, S, M


@dataclass
class Info:
    status: int = OK
    sweeps: int = 0
    lambda_sweeps: int = 0
    rel_res2: float = float("nan")
    res_inf: float = float("nan")
    outer_iters: int = 0


def _check(g, b, x, bnorm):
    r = g.residual(b, x)
    return float(np.linalg.norm(r)) / bnorm, float(np.abs(r).max()) if len(r) else 0.0


def run(g: Graph, b, sweeps, Lt=None, m=None):
    """``sweeps`` iterations from the given (default zero) messages.

    Returns (x, Lt, m): x = read-off of the last iteration, messages after ``sweeps``
    updates.
    """
    Lt = np.zeros(g.E) if Lt is None else Lt
    m = np.zeros(g.E) if m is None else m
    x = None
    for _ in range(sweeps):
        x, Lt, m, _, _ = sweep(g, b, Lt, m)
    return x, Lt, m


def solve(g: Graph, b, tol, max_sweeps, check_every=1, Lt=None, m=None):
    """Algorithm 1, flood schedule, from zero messages. Returns (x, info, Lt, m)."""
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b)) or 1.0
    Lt = np.zeros(g.E) if Lt is None else Lt
    m = np.zeros(g.E) if m is None else m
    info = Info()
    x = np.zeros(g.n)
    for s in range(1, max_sweeps + 1):
        x, Lt, m, S, _ = sweep(g, b, Lt, m)
        if not np.all(np.isfinite(x)):
            info.status, info.sweeps = ENUMERIC, s
            return x, info, Lt, m
        if s % check_every == 0 or s == max_sweeps:
            info.rel_res2, info.res_inf = _check(g, b, x, bnorm)
            info.sweeps = s
            if info.rel_res2 <= tol:
                return x, info, Lt, m
    info.status = MAXSWEEPS
    info.sweeps = max_sweeps
    return x, info, Lt, m


# ----------------------------------------------------------------------------------------
# Precomputed Lambda~ (b-independent), Sec. 2.3 and Sec. 4.2
# ----------------------------------------------------------------------------------------

def lambda_phase(g: Graph, tol_lambda=1e-14, max_sweeps=10000):
    """Iterate the Lt rule alone from zero until max|dLt| <= tol_lambda * max|Lt|.

    Returns (Lt_star, S_star, sweeps): Lt after ``sweeps`` updates and the node precisions
    Sigma built from it. With tol_lambda = 0 exactly ``max_sweeps`` updates are made.
    """
    Lt = np.zeros(g.E)
    zeros = np.zeros(g.n)
    done = 0
    for s in range(1, max_sweeps + 1):
        S, _ = node_totals(g, zeros, Lt, np.zeros(g.E))
        back_L = _gather(Lt, g.rev)
        with np.errstate(divide="ignore", invalid="ignore"):
            Lt_new = -g.a_ij / (S[g.src] - back_L * g.a_ij)
        delta = float(np.abs(Lt_new - Lt).max()) if g.E else 0.0
        scale = float(np.abs(Lt_new).max()) if g.E else 0.0
        Lt = Lt_new
        done = s
        if tol_lambda > 0 and delta <= tol_lambda * scale:
            break
    S_star, _ = node_totals(g, zeros, Lt, np.zeros(g.E))
    return Lt, S_star, done


def msweep(g: Graph, b, Lt_star, S_star, m):
    """One mean-only iteration with frozen Lt*: x = M / S*, m_ji = Lt*_ji (M_j - m_ij)."""
    M = b + np.bincount(g.dst, weights=m, minlength=g.n)
    x = M / S_star
    m_new = Lt_star * (M[g.src] - _gather(m, g.rev))
    return x, m_new


def solve_precomp(g: Graph, b, tol, max_sweeps, check_every=1, tol_lambda=1e-14,
                  max_lambda_sweeps=10000, lam=None):
    """Two-phase solve: Lambda~ once, then mean-only sweeps from zero m."""
    if lam is None:
        Lt_star, S_star, ls = lambda_phase(g, tol_lambda, max_lambda_sweeps)
    else:
        Lt_star, S_star, ls = lam
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b)) or 1.0
    m = np.zeros(g.E)
    info = Info(lambda_sweeps=ls)
    x = np.zeros(g.n)
    for s in range(1, max_sweeps + 1):
        x, m = msweep(g, b, Lt_star, S_star, m)
        if s % check_every == 0 or s == max_sweeps:
            info.rel_res2, info.res_inf = _check(g, b, x, bnorm)
            info.sweeps = s
            if info.rel_res2 <= tol:
                return x, info
    info.status, info.sweeps = MAXSWEEPS, max_sweeps
    return x, info


# ----------------------------------------------------------------------------------------
# Algorithm 3: GaBP as an error-correction smoother
# ----------------------------------------------------------------------------------------

def smooth(g: Graph, b, x, mu, lam=None):
    """x_new = x + e^mu, where e^mu is the mu-th read-off of GaBP on A e = b - A x from zero
    messages (Algorithm 3).

    ``lam=None``: joint sweeps (Algorithm 1 on the error equation). ``lam=(Lt*, S*)``:
    mean-only sweeps with the converged precision messages frozen.
    """
    r = g.residual(b, x)
    m = np.zeros(g.E)
    if lam is None:
        Lt = np.zeros(g.E)
        for _ in range(mu):
            e, Lt, m, _, _ = sweep(g, r, Lt, m)
    else:
        Lt_star, S_star = lam
        for _ in range(mu):
            e, m = msweep(g, r, Lt_star, S_star, m)
    return x + e


def lambda_sequence(g: Graph, depth, colour=None):
    """Precision messages of the first ``depth`` sweeps from zero messages.

    They do not depend on the right-hand side (Sec. 2.3 remark after Algorithm 1), so a
    smoother that restarts from zero messages at every call needs exactly these, and they
    can be computed once and reused by every call (Sec. 4.2, precomputing the required
    messages). Returns ``[(Lt_s, S_s) for s = 1..depth]``: ``S_s`` = the node precisions
    the read-off of sweep s divides by, ``Lt_s`` = the precision messages sent in sweep s.
    ``colour``: the coloured schedule (classes in turn, in place); None: flood.
    """
    seq = []
    Lt = np.zeros(g.E)
    colour = None if colour is None else np.asarray(colour)
    for _ in range(depth):
        if colour is None:
            S, _ = node_totals(g, np.zeros(g.n), Lt, np.zeros(g.E))
            with np.errstate(divide="ignore", invalid="ignore"):
                Lt = -g.a_ij / (S[g.src] - _gather(Lt, g.rev) * g.a_ij)
            seq.append((Lt, S))
            continue
        S_rec = np.zeros(g.n)
        Lt = Lt.copy()
        for c in range(int(colour.max()) + 1 if len(colour) else 0):
            S, _ = node_totals(g, np.zeros(g.n), Lt, np.zeros(g.E))
            sel = colour == c
            S_rec[sel] = S[sel]
            with np.errstate(divide="ignore", invalid="ignore"):
                L_new = -g.a_ij / (S[g.src] - _gather(Lt, g.rev) * g.a_ij)
            Lt = np.where(colour[g.src] == c, L_new, Lt)
        seq.append((Lt.copy(), S_rec))
    return seq


def smooth_seq(g: Graph, b, x, mu, seq, colour=None):
    """Algorithm 3 with mean-only sweeps that take the precision messages of sweep s from
    ``seq = lambda_sequence(g, >= mu, colour)``: the same iterates as the joint smoother
    from zero messages, without recomputing the precision messages."""
    assert len(seq) >= mu
    r = g.residual(b, x)
    m = np.zeros(g.E)
    colour = None if colour is None else np.asarray(colour)
    e = np.zeros(g.n)
    for s in range(mu):
        Lt_s, S_s = seq[s]
        if colour is None:
            M = r + np.bincount(g.dst, weights=m, minlength=g.n)
            e = M / S_s
            m = Lt_s * (M[g.src] - _gather(m, g.rev))
            continue
        for c in range(int(colour.max()) + 1 if len(colour) else 0):
            M = r + np.bincount(g.dst, weights=m, minlength=g.n)
            sel = colour == c
            e[sel] = M[sel] / S_s[sel]
            m_new = Lt_s * (M[g.src] - _gather(m, g.rev))
            m = np.where(colour[g.src] == c, m_new, m)
    return x + e


# ----------------------------------------------------------------------------------------
# FP32 messages inside FP64 iterative refinement
# ----------------------------------------------------------------------------------------

def ir_solve(g: Graph, b, tol, lam32, check_every=16, inner_tol=1e-4, max_inner=10**5,
             max_sweeps=10**6):
    """Classical iterative refinement (not in the paper) around FP32 mean-only GaBP.

    Outer loop in FP64: x = 0; r = b - A x; stop when ||r||_2 / ||b||_2 <= tol. Each outer
    step scales the residual by s = ||r||_inf and solves A d = r / s approximately with
    mean-only sweeps (Sec. 2.3 decoupling) in FP32 from zero messages, using the FP32
    precision messages and reciprocal node precisions ``lam32 = (Lt*, 1/S*)``; the inner
    solve stops when the FP64 residual of the correction equation satisfies
    ||r/s - A d||_2 <= inner_tol ||r/s||_2 (checked every ``check_every`` sweeps) or after
    ``max_inner`` sweeps; then x += s d. Returns MAXSWEEPS when ``max_sweeps`` inner sweeps
    are spent or an outer step does not reduce ||r||_2.
    """
    Lt32, invS32 = lam32
    f32 = np.float32
    x = np.zeros(g.n)
    bnorm = float(np.linalg.norm(b)) or 1.0
    info = Info(status=MAXSWEEPS)
    r = g.residual(b, x)
    prev = np.inf
    while True:
        rn = float(np.linalg.norm(r))
        info.rel_res2, info.res_inf = rn / bnorm, float(np.abs(r).max())
        if info.rel_res2 <= tol:
            info.status = OK
            return x, info
        if info.sweeps >= max_sweeps or not rn < prev:
            return x, info
        prev = rn
        s = float(np.abs(r).max())
        rs = r / s
        r32 = rs.astype(f32)
        m = np.zeros(g.E, dtype=f32)
        inner = 0
        while True:
            for _ in range(check_every):
                M = r32 + np.bincount(g.dst, weights=m, minlength=g.n).astype(f32)
                d = M * invS32
                back = np.where(g.rev >= 0, m[np.maximum(g.rev, 0)], f32(0))
                m = (Lt32 * (M[g.src] - back)).astype(f32)
            inner += check_every
            info.sweeps += check_every
            res = np.linalg.norm(rs - g.matvec(d.astype(np.float64)))
            if (res <= inner_tol * np.linalg.norm(rs) or inner >= max_inner or
                    info.sweeps >= max_sweeps):
                break
        x = x + s * d.astype(np.float64)
        r = g.residual(b, x)
        info.outer_iters += 1


# ----------------------------------------------------------------------------------------
# Red-black schedule (the paper's "red-black GaBP", Sec. 5): Algorithm 1 visiting all red
# nodes, then all black nodes; a visit reads off x_j and sends j's messages, and a node
# of the second colour already receives the messages sent in the first half.
# ----------------------------------------------------------------------------------------

def sweep_coloured(g: Graph, b, Lt, m, colour, lambda_fixed=None):
    """One coloured sweep (red-black, or the 4-colour schedule of Sec. 5): colour classes
    0, 1, ... in turn; each class reads off its nodes and sends their messages from the
    newest messages. colour: a proper colouring (no edge inside a class).

    ``lambda_fixed = (Lt*, S*)``: mean-only with frozen Lambda~ (x = M / S*).
    Returns (x, Lt, m) with x the read-off of each node at its visit.
    """
    colour = np.asarray(colour)
    x = np.zeros(g.n)
    Lt = Lt.copy()
    m = m.copy()
    for c in range(int(colour.max()) + 1 if len(colour) else 0):
        if lambda_fixed is None:
            S, M = node_totals(g, b, Lt, m)
        else:
            S = lambda_fixed[1]
            M = b + np.bincount(g.dst, weights=m, minlength=g.n)
        sel = colour == c
        x[sel] = M[sel] / S[sel]
        upd = colour[g.src] == c
        back_m = _gather(m, g.rev)
        if lambda_fixed is None:
            back_L = _gather(Lt, g.rev)
            with np.errstate(divide="ignore", invalid="ignore"):
                L_new = -g.a_ij / (S[g.src] - back_L * g.a_ij)
            m_new = L_new * (M[g.src] - back_m)
            Lt = np.where(upd, L_new, Lt)
        else:
            m_new = lambda_fixed[0] * (M[g.src] - back_m)
        m = np.where(upd, m_new, m)
    return x, Lt, m


def grid_colour(nx, ny=None):
    """Red-black colouring of an nx x ny grid, x fastest: colour = (ix + iy) mod 2."""
    ny = nx if ny is None else ny
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    return ((ix + iy) % 2).astype(np.uint8)


def grid_colour4(nx, ny=None):
    """Four-colouring of an nx x ny grid proper for 9-point stencils: colour =
    (ix mod 2) + 2 (iy mod 2)."""
    ny = nx if ny is None else ny
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    return ((ix % 2) + 2 * (iy % 2)).astype(np.uint8)


def smooth_coloured(g: Graph, b, x, mu, colour, lam=None):
    """Algorithm 3 with coloured sweeps from zero messages: e^mu = the read-offs of the
    mu-th coloured sweep. ``lam = (Lt*, S*)``: mean-only with the converged precision
    messages frozen; otherwise joint. Returns x + e^mu."""
    r = g.residual(b, x)
    m = np.zeros(g.E)
    Lt = np.zeros(g.E) if lam is None else lam[0]
    for _ in range(mu):
        e, Lt, m = sweep_coloured(g, r, Lt, m, colour, lambda_fixed=lam)
    return x + e
