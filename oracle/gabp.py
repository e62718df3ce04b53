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

def smooth(g: Graph, b, x, mu, lam=None, m_state=None):
    """x_new = x + e^mu, where e^mu is the mu-th read-off of GaBP on A e = b - A x.

    ``lam=None``: joint sweeps from zero messages (Algorithm 1 on the error equation).
    ``lam=(Lt*, S*)``: mean-only sweeps with precomputed Lambda~. ``m_state``: start the
    mean messages from these (warm start) instead of zero; the final messages are returned.
    Returns (x_new, m_after).
    """
    r = g.residual(b, x)
    m = np.zeros(g.E) if m_state is None else m_state.copy()
    if lam is None:
        Lt = np.zeros(g.E)
        for _ in range(mu):
            e, Lt, m, _, _ = sweep(g, r, Lt, m)
    else:
        Lt_star, S_star = lam
        for _ in range(mu):
            e, m = msweep(g, r, Lt_star, S_star, m)
    return x + e, m


# ----------------------------------------------------------------------------------------
# FP32 messages inside FP64 iterative refinement
# ----------------------------------------------------------------------------------------

def ir_solve(g: Graph, b, tol, lam32, check_every=16, inner_tol=1e-4, max_sweeps=10**6,
             patience=8):
    """Iterative refinement with FP32 mean-only GaBP as the inner solver.

    Outer loop in FP64: r = b - A x; stop at ||r||_2/||b||_2 <= tol. Inner: mean-only sweeps
    on A d = r / s (s = ||r||_inf) in FP32 with FP32 Lt*, 1/S*, from zero messages; every
    ``check_every`` sweeps the FP64 residual of x + s d is formed and the best trial kept;
    the inner solve ends when the best trial reached inner_tol * ||r|| or tol * ||b||, or
    after ``patience`` checks without a new best once one was found. Then x += s d_best.
    ``lam32 = (Lt*, 1/S*)`` as float32 arrays. Parity unpinned as a bitwise reference (the
    FP32 rounding order is free); only its converged result is compared.
    """
    Lt32, invS32 = lam32
    f32 = np.float32
    x = np.zeros(g.n)
    bnorm = float(np.linalg.norm(b)) or 1.0
    info = Info(status=MAXSWEEPS)
    r = g.residual(b, x)
    while True:
        rn = float(np.linalg.norm(r))
        info.rel_res2, info.res_inf = rn / bnorm, float(np.abs(r).max())
        if info.rel_res2 <= tol:
            info.status = OK
            return x, info
        if info.sweeps >= max_sweeps:
            return x, info
        s = float(np.abs(r).max())
        r32 = (r / s).astype(f32)
        m = np.zeros(g.E, dtype=f32)
        best, d_best, r_best, since = rn, None, None, 0
        while True:
            for _ in range(check_every):
                M = r32 + np.bincount(g.dst, weights=m, minlength=g.n).astype(f32)
                d = M * invS32
                back = np.where(g.rev >= 0, m[np.maximum(g.rev, 0)], f32(0))
                m = (Lt32 * (M[g.src] - back)).astype(f32)
                info.sweeps += 1
            rt = b - g.matvec(x + s * d.astype(np.float64))
            nt = float(np.linalg.norm(rt))
            if nt < best:
                best, d_best, r_best, since = nt, d.copy(), rt, 0
            else:
                since += 1
            if (best <= inner_tol * rn or best / bnorm <= tol or
                    (d_best is not None and since >= patience) or info.sweeps >= max_sweeps):
                break
        if d_best is None:
            return x, info
        x = x + s * d_best.astype(np.float64)
        r = r_best
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


def smooth_coloured(g: Graph, b, x, mu, colour, lam=None, m_state=None, Lt_state=None):
    """Algorithm 3 with red-black sweeps: e^mu = the read-offs of the mu-th red-black sweep.

    ``lam = (Lt*, S*)``: mean-only with precomputed Lambda~; otherwise joint from
    ``Lt_state`` (zero if None). ``m_state``: warm mean messages. Returns (x_new, Lt, m).
    """
    r = g.residual(b, x)
    m = np.zeros(g.E) if m_state is None else m_state.copy()
    Lt = (np.zeros(g.E) if Lt_state is None else Lt_state.copy()) if lam is None else lam[0]
    for _ in range(mu):
        e, Lt, m = sweep_coloured(g, r, Lt, m, colour, lambda_fixed=lam)
    return x + e, Lt, m
