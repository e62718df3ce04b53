"""Two-layer generalized GaBP (Sec. 3 of arXiv 1904.04093, Algorithm 2) on a region graph
whose small regions are single nodes -- test infrastructure only.

Large regions are index sets of the unknowns. Every small region is one node, and its
parents are the large regions that contain it. Node l receives one scalar precision message
Lambda_{L l} and one scalar mean message m_{L l} from each parent L (the reparametrised
messages of Sec. 3.3: m = Lambda mu). The large regions must cover every off-diagonal
nonzero exactly once (an entry A_ij is "inside" region L when i and j both belong to L).

One iteration, for every large region L, from the messages of the previous iteration
(flood schedule; Algorithm 2 with all regions processed from the same old messages):

* Lambda~_0 = [A]_L + the messages that L's children receive from their other parents
  (added to the diagonal), b~_0 = [b]_L + the matching mean messages;
* [x]_L = Lambda~_0^{-1} b~_0;
* for every child l of L, with s_l = 1 / (Lambda~_0^{-1})_ll:
  Lambda_{L l} = s_l - A_ll - (other parents' Lambda into l),
  m_{L l}      = s_l [x]_l - b_l - (other parents' m into l)
  (eq. Two_layers_GaBP_rules, the form used in Algorithm 2).

The region systems are solved with dense LU (numpy) -- the plain definition; the two-sided
tridiagonal recurrences that a line region allows are deliberately not used here.

Readings of points the paper leaves open (also listed in the design notes):

* initial messages are zero (as for Algorithm 1);
* the read-off is Algorithm 2's own: every region L writes [x]_L = Lambda~_0^{-1} b~_0 when
  it is updated, so a node keeps the solution of the last region containing it in the
  processing order (regions in list order, groups in group order). For the line partition
  (rows listed before columns) that is the node's column solution. ``sweep`` returns it
  with the per-region solutions; ``readoff`` gives the single-node belief
  (b_l + sum m_{L l}) / (A_ll + sum Lambda_{L l}) of a message state instead, which is what
  the Bethe-region reduction to Algorithm 1 compares. At a fixed point both equal A^{-1} b
  (Theorem prop:generalized_GaBP_Consistency);
* Lambda converged: max|dLambda| <= tol_lambda * max|Lambda| between consecutive updates;
* schedules: "flood" (every region from the previous iteration's messages, the literal
  all-regions-in-parallel reading) and, with ``groups``, region groups updated one after
  the other, each from the newest messages. For the line partition the groups are the rows
  and the columns: no two rows share a node (nor two columns), so each group is still
  processed all in parallel, and rows-then-columns is the region-level analogue of the
  red-black point schedule (the region hypergraph is bipartite between rows and columns).

``grid_lines`` builds the line partition of Fig. two_layers_network (horizontal and vertical
stripes of a 2-D grid), which the numerical section calls line GaBP.
"""
from __future__ import annotations

import numpy as np

OK, MAXSWEEPS = 0, 1


class RegionGraph:
    """A square matrix (dense or CSR) and its large regions."""

    def __init__(self, A, regions):
        if hasattr(A, "rowptr"):
            from scipy.sparse import csr_matrix
            self.S = csr_matrix((np.asarray(A.val, float), np.asarray(A.col),
                                 np.asarray(A.rowptr)), shape=(A.n, A.n))
        else:
            from scipy.sparse import csr_matrix
            self.S = csr_matrix(np.asarray(A, dtype=np.float64))
        self.n = self.S.shape[0]
        self.diag = self.S.diagonal().astype(np.float64)
        self.regions = [np.asarray(r, dtype=np.int64) for r in regions]
        # the dense block [A]_L of every region
        self.blocks = [self.S[r][:, r].toarray() for r in self.regions]
        self._check_cover()

    def _check_cover(self):
        coo = self.S.tocoo()
        off = (coo.row != coo.col) & (coo.data != 0)
        count = np.zeros(int(off.sum()), dtype=np.int64)
        rows, cols = coo.row[off], coo.col[off]
        member = np.zeros(self.n, dtype=bool)
        for r in self.regions:
            member[:] = False
            member[r] = True
            count += member[rows] & member[cols]
        if not np.all(count == 1):
            raise ValueError("every off-diagonal nonzero must lie in exactly one large region")

    def zeros(self):
        return [np.zeros(len(r)) for r in self.regions]

    def residual(self, b, x):
        return np.asarray(b, float) - self.S @ np.asarray(x, float)


def grid_lines(nx, ny):
    """Rows (horizontal stripes, y = 0..ny-1) then columns (vertical stripes) of an nx x ny
    grid whose node (x, y) has index y * nx + x."""
    rows = [y * nx + np.arange(nx) for y in range(ny)]
    cols = [x + nx * np.arange(ny) for x in range(nx)]
    return rows + cols


def line_groups(nx, ny):
    """Region groups of ``grid_lines``: all rows, then all columns."""
    return [list(range(ny)), list(range(ny, ny + nx))]


def edge_regions(A):
    """The Bethe regions: one large region {i, j} per pair with A_ij != 0 or A_ji != 0.

    With these regions the two-layer rules reduce to ordinary GaBP (end of Sec. 3.2)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    regs = []
    for i in range(n):
        for j in range(i + 1, n):
            if A[i, j] != 0 or A[j, i] != 0:
                regs.append([i, j])
    return regs


def _totals(rg, lam, m):
    tl = np.zeros(rg.n)
    tm = np.zeros(rg.n)
    for r, lk, mk in zip(rg.regions, lam, m):
        np.add.at(tl, r, lk)
        np.add.at(tm, r, mk)
    return tl, tm


def readoff(rg, b, lam, m):
    """Belief of every single-node region from all its incoming messages."""
    tl, tm = _totals(rg, lam, m)
    return (np.asarray(b, float) + tm) / (rg.diag + tl)


def sweep(rg, b, lam, m, lam_fixed=None, groups=None):
    """One iteration. Returns (x, x_regions, lam_new, m_new).

    x_regions[k] = [x]_L of region k computed in this iteration; x is Algorithm 2's read-off
    (every node takes the [x]_L of the last region written that contains it). ``lam_fixed = (lam*, inverses)`` freezes the precision messages and
    reuses the region inverses (precomputed Lambda, Sec. 4.2 applied to Algorithm 2).
    ``groups`` (lists of region indices): update group by group from the newest messages;
    None: flood, every region from the incoming messages.
    """
    b = np.asarray(b, dtype=np.float64)
    tl, tm = _totals(rg, lam, m)
    x = np.full(rg.n, np.nan)
    lam_new, m_new = list(lam), list(m)
    xr = [None] * len(rg.regions)
    for grp in (groups if groups is not None else [range(len(rg.regions))]):
        if groups is not None:
            tl, tm = _totals(rg, lam_new, m_new)
        upd = []
        for k in grp:
            r = rg.regions[k]
            other_l = tl[r] - lam_new[k]
            other_m = tm[r] - m_new[k]
            if lam_fixed is None:
                inv = np.linalg.inv(rg.blocks[k] + np.diag(other_l))
            else:
                inv = lam_fixed[1][k]
            xl = inv @ (b[r] + other_m)
            s = 1.0 / np.diag(inv)
            upd.append((k, s - rg.diag[r] - other_l if lam_fixed is None else lam[k],
                        s * xl - b[r] - other_m))
            xr[k] = xl
            x[r] = xl
        for k, lk, mk in upd:
            lam_new[k], m_new[k] = lk, mk
    # nodes in no region keep the belief of their (message-free) small region
    lone = np.isnan(x)
    x[lone] = b[lone] / rg.diag[lone]
    return x, xr, lam_new, m_new


def run(rg, b, sweeps, lam=None, m=None, groups=None):
    """``sweeps`` iterations from the given (default zero) messages: (x, lam, m)."""
    lam = rg.zeros() if lam is None else lam
    m = rg.zeros() if m is None else m
    x = None
    for _ in range(sweeps):
        x, _, lam, m = sweep(rg, b, lam, m, groups=groups)
    return x, lam, m


def lambda_phase(rg, tol_lambda=1e-14, max_sweeps=10000, groups=None):
    """Iterate the precision messages alone from zero (they do not depend on b).

    Returns (lam*, inverses, sweeps): the messages after ``sweeps`` updates and the region
    inverses (Lambda~_0)^{-1} built from them, which the frozen mean iteration reuses."""
    lam = rg.zeros()
    zb = np.zeros(rg.n)
    done = 0
    for s in range(1, max_sweeps + 1):
        _, _, new, _ = sweep(rg, zb, lam, rg.zeros(), groups=groups)
        flat_new = np.concatenate(new) if new else np.zeros(0)
        flat_old = np.concatenate(lam) if lam else np.zeros(0)
        delta = float(np.abs(flat_new - flat_old).max()) if len(flat_new) else 0.0
        scale = float(np.abs(flat_new).max()) if len(flat_new) else 0.0
        lam = new
        done = s
        if tol_lambda > 0 and delta <= tol_lambda * scale:
            break
    tl, _ = _totals(rg, lam, rg.zeros())
    invs = [np.linalg.inv(rg.blocks[k] + np.diag(tl[r] - lam[k]))
            for k, r in enumerate(rg.regions)]
    return lam, invs, done


def solve(rg, b, tol, max_sweeps, check_every=1, precomp=None, groups=None):
    """Sweeps until ||b - A x||_2 / ||b||_2 <= tol at a check. ``precomp = (lam*, inverses)``
    runs the mean-only iteration. Returns (x, status, sweeps, rel_res)."""
    b = np.asarray(b, dtype=np.float64)
    bn = float(np.linalg.norm(b)) or 1.0
    lam = rg.zeros() if precomp is None else precomp[0]
    m = rg.zeros()
    rel = float("nan")
    x = np.zeros(rg.n)
    for s in range(1, max_sweeps + 1):
        x, _, lam, m = sweep(rg, b, lam, m, lam_fixed=precomp, groups=groups)
        if s % check_every == 0 or s == max_sweeps:
            rel = float(np.linalg.norm(rg.residual(b, x))) / bn
            if rel <= tol:
                return x, OK, s, rel
    return x, MAXSWEEPS, max_sweeps, rel


def smooth(rg, b, x, mu, precomp=None, groups=None):
    """Algorithm 3 with the region iteration: x + (mu-th read-off of the sweeps on
    A e = b - A x from zero messages). ``precomp = (lam*, inverses)`` freezes the converged
    precision messages."""
    r = rg.residual(b, x)
    lam = rg.zeros() if precomp is None else precomp[0]
    m = rg.zeros()
    e = None
    for _ in range(mu):
        e, _, lam, m = sweep(rg, r, lam, m, lam_fixed=precomp, groups=groups)
    return np.asarray(x, float) + e
