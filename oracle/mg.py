"""Geometric multigrid V-cycle with GaBP or red-black Gauss-Seidel smoothing
(test infrastructure only).

Sec. 4 of the paper: a two-grid cycle applied recursively (V-cycle); grids with 2^J + 1
points per side including the boundary, the coarse grid keeping every second point;
full-weighting restriction and bilinear interpolation (the Trottenberg et al. operators the
paper cites); the coarse operators are finite-difference rediscretisations (supplied by the
caller); the coarsest system is solved directly (LU). GaBP enters as the error-correction
smoother of Algorithm 3; red-black Gauss-Seidel is the classical comparison smoother of the
numerical section.

Grids are vertex-centred with n x n interior nodes and n = 2 n_c + 1; coarse interior node
(I, J) sits on fine interior node (2I+1, 2J+1). Arrays are flat, x fastest.
"""
from __future__ import annotations

import numpy as np

from . import gabp as _g
from . import regions as _rg


def restrict_fw(r, n_f):
    """Full weighting: stencil [1 2 1; 2 4 2; 1 2 1] / 16 centred on the coarse points."""
    n_c = (n_f - 1) // 2
    R = np.asarray(r, dtype=np.float64).reshape(n_f, n_f)
    c = 4.0 * R[1::2, 1::2]
    c += 2.0 * (R[0:-1:2, 1::2] + R[2::2, 1::2] + R[1::2, 0:-1:2] + R[1::2, 2::2])
    c += R[0:-1:2, 0:-1:2] + R[0:-1:2, 2::2] + R[2::2, 0:-1:2] + R[2::2, 2::2]
    assert c.shape == (n_c, n_c)
    return (c / 16.0).reshape(-1)


def prolong_bilinear(e_c, n_c):
    """Bilinear interpolation from the coarse interior grid (zero Dirichlet boundary)."""
    n_f = 2 * n_c + 1
    E = np.zeros((n_c + 2, n_c + 2))
    E[1:-1, 1:-1] = np.asarray(e_c, dtype=np.float64).reshape(n_c, n_c)
    F = np.zeros((n_f + 2, n_f + 2))
    F[::2, ::2] = E
    F[::2, 1::2] = 0.5 * (E[:, :-1] + E[:, 1:])
    F[1::2, :] = 0.5 * (F[0:-1:2, :] + F[2::2, :])
    return F[1:-1, 1:-1].reshape(-1)


def rbgs(g: _g.Graph, b, x, n, sweeps):
    """Red-black Gauss-Seidel on an n x n grid; red = (ix + iy) even, updated first."""
    x = np.array(x, dtype=np.float64)
    iy, ix = np.divmod(np.arange(g.n), n)
    colour = (ix + iy) % 2
    off = g.rows != g.cols
    for _ in range(sweeps):
        for c in (0, 1):
            sel = colour == c
            s = np.bincount(g.rows[off], weights=g.vals[off] * x[g.cols[off]], minlength=g.n)
            x[sel] = (b[sel] - s[sel]) / g.diag[sel]
    return x


class Hierarchy:
    """Per-level oracle state: graphs, grid sides and precomputed precision messages.

    smoother: "rbgs" (red-black Gauss-Seidel) or "gabp" (Algorithm 3, messages restarted
    from zero at every call) with gabp_mode "joint" (precision messages recomputed every
    sweep), "precomp" (the converged precision messages frozen) or "seq" (the precision
    messages of the smoother's own sweeps precomputed once: the same iterates as "joint"),
    and schedule "flood" | "redblack" | "colour4" | "lines" | "lines_alt". "lines" is the
    two-layer region iteration on the grid's rows and columns (Algorithm 2 with the
    partition of Fig. two_layers_network, line GaBP) in the flood schedule; "lines_alt"
    updates all rows, then all columns.
    """

    def __init__(self, csrs, smoother="gabp", nu1=2, nu2=2, gabp_mode="precomp",
                 tol_lambda=1e-14, max_lambda_sweeps=10000, schedule="flood"):
        self.graphs = [_g.Graph.from_csr(a) for a in csrs]
        self.sides = [int(round(np.sqrt(a.n))) for a in csrs]
        self.smoother, self.nu1, self.nu2 = smoother, nu1, nu2
        self.gabp_mode, self.schedule = gabp_mode, schedule
        self.lam = [None] * len(csrs)
        self.seq = [None] * len(csrs)
        self.rgs = None
        if smoother == "gabp" and schedule in ("lines", "lines_alt"):
            if gabp_mode == "seq":
                raise ValueError("per-sweep precision messages are built for point schedules")
            self.rgs = [_rg.RegionGraph(a, _rg.grid_lines(s, s))
                        for a, s in zip(csrs[:-1], self.sides[:-1])]
            self.groups = [None if schedule == "lines" else _rg.line_groups(s, s)
                           for s in self.sides[:-1]]
            if gabp_mode == "precomp":
                for l, rg in enumerate(self.rgs):
                    lam, invs, _ = _rg.lambda_phase(rg, tol_lambda, max_lambda_sweeps,
                                                    groups=self.groups[l])
                    self.lam[l] = (lam, invs)
        elif smoother == "gabp" and gabp_mode == "precomp":
            for l, g in enumerate(self.graphs[:-1]):
                Lt, S, _ = _g.lambda_phase(g, tol_lambda, max_lambda_sweeps)
                self.lam[l] = (Lt, S)
        elif smoother == "gabp" and gabp_mode == "seq":
            for l, g in enumerate(self.graphs[:-1]):
                self.seq[l] = _g.lambda_sequence(g, max(nu1, nu2, 1), self._colour(l))
        self.coarse = np.linalg.inv(self.graphs[-1].dense())

    def _colour(self, l):
        if self.schedule == "redblack":
            return _g.grid_colour(self.sides[l])
        if self.schedule == "colour4":
            return _g.grid_colour4(self.sides[l])
        return None

    def _smooth(self, l, b, x, nu):
        g = self.graphs[l]
        if nu == 0:
            return x
        if self.smoother == "rbgs":
            return rbgs(g, b, x, self.sides[l], nu)
        if self.schedule in ("lines", "lines_alt"):
            return _rg.smooth(self.rgs[l], b, x, nu, precomp=self.lam[l], groups=self.groups[l])
        col = self._colour(l)
        if self.seq[l] is not None:
            return _g.smooth_seq(g, b, x, nu, self.seq[l], col)
        if col is not None:
            return _g.smooth_coloured(g, b, x, nu, col, lam=self.lam[l])
        return _g.smooth(g, b, x, nu, lam=self.lam[l])

    def vcycle(self, b, x, l=0):
        """One V(nu1, nu2) cycle on level l; returns the new iterate."""
        g = self.graphs[l]
        if l == len(self.graphs) - 1:
            return self.coarse @ b
        x = self._smooth(l, b, x, self.nu1)
        r = g.residual(b, x)
        rc = restrict_fw(r, self.sides[l])
        ec = self.vcycle(rc, np.zeros(self.graphs[l + 1].n), l + 1)
        x = x + prolong_bilinear(ec, self.sides[l + 1])
        return self._smooth(l, b, x, self.nu2)

    def solve(self, b, tol, max_cycles):
        g = self.graphs[0]
        x = np.zeros(g.n)
        bn = float(np.linalg.norm(b)) or 1.0
        hist = []
        for k in range(max_cycles):
            x = self.vcycle(b, x)
            rel = float(np.linalg.norm(g.residual(b, x))) / bn
            hist.append(rel)
            if rel <= tol or not np.isfinite(rel):
                break
        return x, hist
