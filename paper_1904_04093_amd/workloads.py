"""Seeded synthetic inputs for the GaBP solver.

This module only *generates inputs*: sparse matrices in CSR form, right-hand sides and the
random numbers behind them. It holds none of the belief-propagation arithmetic, so both the
HIP path and the CPU oracle can take their inputs from here without sharing any of the
method.

Operators are 2-D second-order elliptic finite-difference operators on the unit square with
homogeneous Dirichlet boundaries, the family the paper's numerical section works with
(Sec. 5; the stand-alone problem there mixes second-order diffusion with first-order
convection):

    -div(k grad u) + v . grad u = f        on (0,1)^2,  u = 0 on the boundary.

Discretisation (the paper leaves it unstated; this is the reading used throughout):

* vertex-centred grid with ``n x n`` interior nodes, ``h = 1/(n+1)``, node ``(ix, iy)`` at
  ``((ix+1) h, (iy+1) h)``, row index ``i = iy * n + ix`` (x fastest);
* 5-point diffusion with face coefficients ``k`` taken at face midpoints;
* first-order upwind convection chosen by the sign of ``v`` at the node;
* rows scaled by ``h^2`` (``scaled=True``) or not; GaBP iterates are invariant under row
  scaling, so the scaling only changes the units of ``b``.

Every upwind operator built here is an M-matrix (non-positive off-diagonals, weakly
diagonally dominant, irreducible), so flood GaBP converges on it (the paper's corollary to
its convergence theorem, Sec. 2.3).

Seeds: ``numpy.random.default_rng(SeedSequence([cfg, sub, ...]))``; see ``rng``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng", "CSR", "assemble_cd", "random_field", "eval_field",
    "small_upwind", "precision_at_scale", "batch_family", "anisotropic_mg",
    "mg_hierarchy", "theta_problem", "theta_jacobian",
    "random_walk_summable", "random_tridiagonal", "manufactured_solution", "random_tree", "laplacian_5pt",
    "toy_5x5", "csr_from_dense", "csr_to_dense", "grid_colouring", "random_sparse_dominant",
]


def rng(*key: int) -> np.random.Generator:
    """Counter-style seeding: one independent stream per integer key tuple."""
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


@dataclass
class CSR:
    """Square CSR matrix, int32 indices, float64 values, columns sorted within rows."""
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_of_nnz(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.rowptr))

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """Plain y = A x (used by generators for manufactured right-hand sides)."""
        rows = self.row_of_nnz()
        y = np.zeros(self.n, dtype=np.result_type(self.val, x))
        np.add.at(y, rows, self.val * x[self.col])
        return y


def csr_from_dense(a: np.ndarray, meta: dict | None = None) -> CSR:
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    rows, cols = np.nonzero(a)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return CSR(n, rowptr, cols.astype(np.int32), a[rows, cols].copy(), dict(meta or {}))


def csr_to_dense(a: CSR) -> np.ndarray:
    d = np.zeros((a.n, a.n))
    d[a.row_of_nnz(), a.col] = a.val
    return d


# ----------------------------------------------------------------------------------------
# Grid operators
# ----------------------------------------------------------------------------------------

def assemble_cd(n: int, kx_face: np.ndarray, ky_face: np.ndarray, vx: np.ndarray,
                vy: np.ndarray, *, scaled: bool = True, with_index: bool = False):
    """Upwind convection-diffusion on an ``n x n`` interior grid.

    ``kx_face[iy, f]`` (shape ``(n, n+1)``) is the coefficient on the x-face between
    ``ix = f-1`` and ``ix = f`` (``f = 0`` and ``f = n`` are boundary faces);
    ``ky_face[f, ix]`` (shape ``(n+1, n)``) likewise for y-faces. ``vx, vy`` are ``(n, n)``
    node velocities. Returns a CSR whose rows list columns in the order
    S (i-n), W (i-1), diagonal, E (i+1), N (i+n).
    With ``with_index`` also returns ``pos[i, t]``: the nnz index of slot ``t`` of row ``i``
    in that S, W, D, E, N order (-1 where the neighbour is outside the grid).
    """
    h = 1.0 / (n + 1)
    kx_face = np.asarray(kx_face, dtype=np.float64)
    ky_face = np.asarray(ky_face, dtype=np.float64)
    vx = np.asarray(vx, dtype=np.float64)
    vy = np.asarray(vy, dtype=np.float64)
    assert kx_face.shape == (n, n + 1) and ky_face.shape == (n + 1, n)
    assert vx.shape == (n, n) and vy.shape == (n, n)
    kw, ke = kx_face[:, :-1], kx_face[:, 1:]
    ks, kn = ky_face[:-1, :], ky_face[1:, :]
    cpx, cmx = h * np.maximum(vx, 0.0), h * np.maximum(-vx, 0.0)
    cpy, cmy = h * np.maximum(vy, 0.0), h * np.maximum(-vy, 0.0)
    diag = kw + ke + ks + kn + cpx + cmx + cpy + cmy
    coef = np.stack([-(ks + cpy), -(kw + cpx), diag, -(ke + cmx), -(kn + cmy)], axis=-1)
    if not scaled:
        coef = coef / (h * h)
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    exists = np.stack([iy > 0, ix > 0, np.ones_like(ix, bool), ix < n - 1, iy < n - 1], -1)
    idx = (iy * n + ix)[..., None] + np.array([-n, -1, 0, 1, n])
    exists = exists.reshape(n * n, 5)
    cols = idx.reshape(n * n, 5)[exists].astype(np.int32)
    vals = coef.reshape(n * n, 5)[exists]
    counts = exists.sum(1)
    rowptr = np.zeros(n * n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(counts)
    a = CSR(n * n, rowptr, cols, vals, {"grid": (n, n), "h": h, "scaled": scaled})
    if with_index:
        pos = np.full(n * n * 5, -1, dtype=np.int64)
        pos[exists.reshape(-1)] = np.arange(rowptr[-1])
        return a, pos.reshape(n * n, 5)
    return a


def _grid_xy(n: int):
    h = 1.0 / (n + 1)
    t = (np.arange(n) + 1) * h
    y, x = np.meshgrid(t, t, indexing="ij")  # [iy, ix]
    return x, y, h


def _face_xy(n: int):
    """Midpoints of x-faces (n, n+1) and y-faces (n+1, n)."""
    h = 1.0 / (n + 1)
    xf = (np.arange(n + 1) + 0.5) * h
    yc = (np.arange(n) + 1) * h
    yfx, xfx = np.meshgrid(yc, xf, indexing="ij")
    yf = (np.arange(n + 1) + 0.5) * h
    xc = (np.arange(n) + 1) * h
    yfy, xfy = np.meshgrid(yf, xc, indexing="ij")
    return (xfx, yfx), (xfy, yfy)


def random_field(r: np.random.Generator, modes: int = 16, kmax: int = 8):
    """Smooth random field g = sum_m a_m cos(2 pi (p_m x + q_m y) + phi_m).

    Wavenumbers p_m, q_m uniform on {1..kmax}, phases uniform, amplitudes uniform and
    normalised so that sum |a_m| = 1 (hence exp(g) lies in [1/e, e]).
    """
    p = r.integers(1, kmax + 1, size=modes)
    q = r.integers(1, kmax + 1, size=modes)
    phi = r.uniform(0.0, 2 * np.pi, size=modes)
    a = r.uniform(-1.0, 1.0, size=modes)
    a = a / np.abs(a).sum()
    return a, p, q, phi


def eval_field(params, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    a, p, q, phi = params
    g = np.zeros(np.broadcast(x, y).shape)
    for m in range(len(a)):
        g += a[m] * np.cos(2 * np.pi * (p[m] * x + q[m] * y) + phi[m])
    return g


def _rotating(n: int, scale: float):
    x, y, _ = _grid_xy(n)
    return -scale * (y - 0.5), scale * (x - 0.5)


def small_upwind(n: int = 32, vx: float = 16.5, vy: float = 8.25, seed=(1, 0)):
    """Constant-coefficient upwind operator (k = 1, constant v), ``b = h^2 f``, f ~ U(-1,1).

    At n = 32 this is the 1024-unknown, 4992-nonzero case: diag 4.75, W -1.5, E -1,
    S -1.25, N -1 (cell Peclet 0.5 in x, 0.25 in y).
    """
    h = 1.0 / (n + 1)
    a = assemble_cd(n, np.ones((n, n + 1)), np.ones((n + 1, n)),
                    np.full((n, n), float(vx)), np.full((n, n), float(vy)))
    f = rng(*seed).uniform(-1.0, 1.0, size=n * n)
    a.meta.update(name=f"upwind{n}", v=(vx, vy))
    return a, h * h * f


def _field_operator(n: int, g_params, vscale: float = 20.0, kx: float = 1.0, ky: float = 1.0,
                    scaled: bool = True):
    (xfx, yfx), (xfy, yfy) = _face_xy(n)
    kxf = kx * np.exp(eval_field(g_params, xfx, yfx))
    kyf = ky * np.exp(eval_field(g_params, xfy, yfy))
    vx, vy = _rotating(n, vscale)
    return assemble_cd(n, kxf, kyf, vx, vy, scaled=scaled)


def precision_at_scale(n: int = 2048, seed: int = 2):
    """Variable diffusion k = exp(g), rotating v = 20(-(y-1/2), x-1/2), b ~ U(-1,1)."""
    g = random_field(rng(seed, 0))
    a = _field_operator(n, g)
    b = rng(seed, 1).uniform(-1.0, 1.0, size=n * n)
    a.meta.update(name=f"cd_field{n}")
    return a, b


def batch_family(nsys: int = 512, nrhs: int = 4, side_lo: int = 48, side_hi: int = 384,
                 seed: int = 3):
    """Independent systems of the variable-coefficient family with uneven grid sides.

    Returns a list of (CSR, B) with B of shape (nrhs, side^2), each U(-1,1).
    """
    sides = rng(seed, 0).integers(side_lo, side_hi + 1, size=nsys)
    out = []
    for t, s in enumerate(sides):
        g = random_field(rng(seed, 1, t))
        a = _field_operator(int(s), g)
        bb = rng(seed, 2, t).uniform(-1.0, 1.0, size=(nrhs, int(s) * int(s)))
        out.append((a, bb))
    return out


def manufactured_solution(a: CSR, n: int, seed: int = 2):
    """Smooth manufactured solution x* on the ``n x n`` grid of ``a`` (a 16-mode random field
    like the coefficient field, stream [seed, 2]) and the right-hand side b := A x*, so that
    the error of a computed x is known exactly."""
    x, y, _ = _grid_xy(n)
    xs = eval_field(random_field(rng(seed, 2)), x, y).reshape(-1)
    rows = a.row_of_nnz()
    return xs, np.bincount(rows, weights=a.val * xs[a.col], minlength=a.n)


def anisotropic_mg(n: int, kx: float = 1.0, ky: float = 0.01, peclet: float = 4.0,
                   h_fine: float | None = None, scaled: bool = False):
    """Anisotropic upwind operator on an ``n x n`` interior grid.

    Diffusion kx (x) and ky (y); rotating velocity scaled so that the cell Peclet number
    max(|vx| h/kx, |vy| h/ky) equals ``peclet`` on the grid with spacing ``h_fine``
    (default: this grid). Coarse grids built with the finest grid's ``h_fine`` therefore see
    the same continuous velocity field and larger cell Peclet numbers.
    """
    h = 1.0 / (n + 1)
    hf = h if h_fine is None else h_fine
    c = peclet / (0.5 * hf * max(1.0 / kx, 1.0 / ky))
    vx, vy = _rotating(n, c)
    return assemble_cd(n, np.full((n, n + 1), kx), np.full((n + 1, n), ky), vx, vy,
                       scaled=scaled)


def mg_hierarchy(J: int, coarsest: int = 3, **kw):
    """Rediscretised operators on nested vertex-centred grids, finest first.

    Level l has 2^l - 1 interior points per side (2^l + 1 with the boundary); the coarse
    grid keeps every second point. Operators are unscaled (no h^2 factor), so restricted
    residuals need no rescaling between levels.
    """
    n_f = 2 ** J - 1
    h_f = 1.0 / (n_f + 1)
    levels = []
    lvl = J
    while True:
        n = 2 ** lvl - 1
        levels.append(anisotropic_mg(n, h_fine=h_f, scaled=False, **kw))
        if n <= coarsest:
            break
        lvl -= 1
    return levels


def theta_problem(n: int, t: int, seed: int = 5, vscale: float = 20.0):
    """Per-node log-diffusion field theta_t (a smooth random field sampled at nodes)."""
    g = random_field(rng(seed, t))
    x, y, _ = _grid_xy(n)
    return eval_field(g, x, y).reshape(-1)


def _theta_faces(n: int, theta: np.ndarray):
    th = np.asarray(theta, dtype=np.float64).reshape(n, n)
    kxf = np.empty((n, n + 1))
    kxf[:, 1:-1] = np.exp(0.5 * (th[:, :-1] + th[:, 1:]))
    kxf[:, 0] = np.exp(th[:, 0])
    kxf[:, -1] = np.exp(th[:, -1])
    kyf = np.empty((n + 1, n))
    kyf[1:-1, :] = np.exp(0.5 * (th[:-1, :] + th[1:, :]))
    kyf[0, :] = np.exp(th[0, :])
    kyf[-1, :] = np.exp(th[-1, :])
    return kxf, kyf


def theta_operator(n: int, theta: np.ndarray, vscale: float = 20.0, with_index=False):
    """A(theta): face coefficient exp((theta_a + theta_b)/2), boundary faces exp(theta_a)."""
    kxf, kyf = _theta_faces(n, theta)
    vx, vy = _rotating(n, vscale)
    return assemble_cd(n, kxf, kyf, vx, vy, with_index=with_index)


def theta_jacobian(n: int, theta: np.ndarray, vscale: float = 20.0):
    """Sparse derivative dA_e/dtheta_p of ``theta_operator`` (e = nnz index, p = node).

    Returned parameter-major: ``(jptr[n*n+1], jnnz[...], jw[...])`` so that
    ``dL/dtheta_p = sum_k jw[k] * G[jnnz[k]]`` for k in ``jptr[p]:jptr[p+1]``, where
    ``G_e = dL/dA_e``. Derivative of the problem definition, not of the solver.
    """
    a, pos = theta_operator(n, theta, vscale, with_index=True)
    kxf, kyf = _theta_faces(n, theta)
    N = n * n
    rows, cols, ws = [], [], []   # (param, nnz index, weight)
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    node = (iy * n + ix)
    # slot order in pos: 0 S, 1 W, 2 D, 3 E, 4 N
    # interior x-faces between (iy, ix) and (iy, ix+1): k = kxf[iy, ix+1]
    for (a_sel, b_sel, k, ab_slot, ba_slot) in (
            ((slice(None), slice(0, n - 1)), (slice(None), slice(1, n)), kxf[:, 1:-1], 3, 1),
            ((slice(0, n - 1), slice(None)), (slice(1, n), slice(None)), kyf[1:-1, :], 4, 0)):
        pa = node[a_sel].reshape(-1)
        pb = node[b_sel].reshape(-1)
        kk = k.reshape(-1)
        for p in (pa, pb):
            for e, s in ((pos[pa, 2], 1.0), (pos[pb, 2], 1.0),
                         (pos[pa, ab_slot], -1.0), (pos[pb, ba_slot], -1.0)):
                rows.append(p)
                cols.append(e)
                ws.append(0.5 * s * kk)
    # boundary faces: k = exp(theta_a), only the diagonal of a
    bx = [(node[:, 0], kxf[:, 0]), (node[:, -1], kxf[:, -1]),
          (node[0, :], kyf[0, :]), (node[-1, :], kyf[-1, :])]
    for p, k in bx:
        rows.append(p)
        cols.append(pos[p, 2])
        ws.append(k.copy())
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    w = np.concatenate(ws)
    assert (c >= 0).all()
    key = r * (a.nnz + 1) + c
    order = np.argsort(key, kind="stable")
    key, r, c, w = key[order], r[order], c[order], w[order]
    uniq, start = np.unique(key, return_index=True)
    wsum = np.add.reduceat(w, start)
    r, c = r[start], c[start]
    jptr = np.zeros(N + 1, dtype=np.int32)
    np.add.at(jptr, r + 1, 1)
    jptr = np.cumsum(jptr).astype(np.int32)
    return a, jptr, c.astype(np.int32), wsum


# ----------------------------------------------------------------------------------------
# Small structured test matrices
# ----------------------------------------------------------------------------------------

def laplacian_5pt(n: int) -> CSR:
    """The 5-point Laplacian [ -1; -1 4 -1; -1 ] on an n x n interior grid (h^2 scaled)."""
    return assemble_cd(n, np.ones((n, n + 1)), np.ones((n + 1, n)), np.zeros((n, n)),
                       np.zeros((n, n)))


def random_walk_summable(n: int, density: float, r: np.random.Generator,
                         margin: float = 0.3, symmetric_pattern: bool = False) -> CSR:
    """Random nonsymmetric matrix with rho(|R|) < 1 by strict row dominance.

    Off-diagonals of random sign; A_ii = +-(1+margin) * sum_j |A_ij| (random sign), so the
    sufficient condition of the paper's convergence theorem holds.
    """
    mask = r.random((n, n)) < density
    if symmetric_pattern:
        mask = mask | mask.T
    np.fill_diagonal(mask, False)
    a = np.where(mask, r.uniform(-1.0, 1.0, (n, n)), 0.0)
    s = np.abs(a).sum(1)
    s[s == 0] = 1.0
    sign = np.where(r.random(n) < 0.5, -1.0, 1.0)
    np.fill_diagonal(a, sign * (1.0 + margin) * s)
    return csr_from_dense(a)


def random_tridiagonal(n: int, r: np.random.Generator) -> CSR:
    """Nonsymmetric tridiagonal matrix with independent random sub/super diagonals."""
    sgn = lambda k: np.where(r.random(k) < 0.5, -1.0, 1.0)
    a = np.diag(r.uniform(2.0, 2.5, n) * sgn(n))
    a += np.diag(r.uniform(0.5, 1.0, n - 1) * sgn(n - 1), 1)
    a += np.diag(r.uniform(0.5, 1.0, n - 1) * sgn(n - 1), -1)
    return csr_from_dense(a)


def random_tree(n: int, r: np.random.Generator, one_way: float = 0.0):
    """Matrix whose (undirected) graph is a random tree.

    With probability ``one_way`` a tree edge keeps only one of A_ij, A_ji (structurally
    nonsymmetric). Returns (CSR, parent array).
    """
    parent = np.full(n, -1)
    a = np.zeros((n, n))
    for v in range(1, n):
        p = int(r.integers(0, v))
        parent[v] = p
        u1, u2 = r.uniform(-1.0, 1.0, 2)
        if r.random() < one_way:
            if r.random() < 0.5:
                u1 = 0.0
            else:
                u2 = 0.0
        a[v, p] = u1
        a[p, v] = u2
    np.fill_diagonal(a, r.uniform(2.0, 3.0, n) * np.where(r.random(n) < 0.5, -1, 1))
    return csr_from_dense(a), parent


def toy_5x5(r: np.random.Generator) -> CSR:
    """Random values on the 5x5 tree pattern of Sec. 2.1 (edges 1-3, 2-3, 3-5, 4-5)."""
    pat = np.array([[1, 0, 1, 0, 0],
                    [0, 1, 1, 0, 0],
                    [1, 1, 1, 0, 1],
                    [0, 0, 0, 1, 1],
                    [0, 0, 1, 1, 1]], dtype=bool)
    a = np.where(pat, r.uniform(-1.0, 1.0, (5, 5)), 0.0)
    np.fill_diagonal(a, r.uniform(3.0, 4.0, 5))
    return csr_from_dense(a)


def grid_colouring(n: int) -> np.ndarray:
    """Red-black colouring of the n x n grid (x fastest): 0 where ix + iy is even."""
    iy, ix = np.divmod(np.arange(n * n), n)
    return ((ix + iy) & 1).astype(np.uint8)


def random_grid_9pt(nx: int, ny: int, r: np.random.Generator, margin: float = 0.2,
                    flip: float = 0.1) -> CSR:
    """Random 9-point operator on an nx x ny grid (node (x, y) has index y * nx + x):
    couplings of magnitude U(0.2, 1), negative except a fraction ``flip``, diagonal
    (1 + margin) times the row's absolute off-diagonal sum."""
    n = nx * ny
    iy, ix = np.divmod(np.arange(n), nx)
    offs = [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]
    coef = -r.uniform(0.2, 1.0, (n, 9)) * np.where(r.random((n, 9)) < flip, -1.0, 1.0)
    exists = np.stack([(ix + dx >= 0) & (ix + dx < nx) & (iy + dy >= 0) & (iy + dy < ny)
                       for dx, dy in offs], -1)
    coef = np.where(exists, coef, 0.0)
    coef[:, 4] = 0.0
    coef[:, 4] = (1.0 + margin) * np.abs(coef).sum(1)
    cols = (np.arange(n)[:, None] + np.array([dy * nx + dx for dx, dy in offs]))[exists]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(exists.sum(1))
    return CSR(n, rowptr, cols.astype(np.int32), coef[exists], {"grid": (nx, ny)})


def grid_colouring4(n: int) -> np.ndarray:
    """Four-colouring of the n x n grid (x fastest) that is proper for 9-point stencils:
    (ix mod 2) + 2 (iy mod 2)."""
    iy, ix = np.divmod(np.arange(n * n), n)
    return ((ix & 1) + 2 * (iy & 1)).astype(np.uint8)


def random_sparse_dominant(n: int, per_row: int, r: np.random.Generator,
                           margin: float = 0.3) -> CSR:
    """Sparse nonsymmetric matrix with ``per_row`` random off-diagonals per row (arbitrary,
    long-range columns) and a strictly dominant diagonal, built without a dense array."""
    rows = np.repeat(np.arange(n), per_row)
    cols = r.integers(0, n, size=n * per_row)
    keep = cols != rows
    rows, cols = rows[keep], cols[keep]
    key = np.unique(rows.astype(np.int64) * n + cols)
    rows, cols = (key // n).astype(np.int64), (key % n).astype(np.int64)
    vals = r.uniform(-1.0, 1.0, size=len(rows))
    s = np.bincount(rows, weights=np.abs(vals), minlength=n)
    s[s == 0] = 1.0
    d = np.where(r.random(n) < 0.5, -1.0, 1.0) * (1.0 + margin) * s
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, np.arange(n)])
    vals = np.concatenate([vals, d])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(np.bincount(rows, minlength=n))
    return CSR(n, rowptr, cols.astype(np.int32), vals)


def random_grid_5pt(nx: int, ny: int, r: np.random.Generator, margin: float = 0.3,
                    kx: float = 1.0, ky: float = 1.0, one_way: float = 0.0,
                    flip: float = 0.0) -> CSR:
    """Random 5-point operator on an nx x ny grid (node (x, y) has index y * nx + x; rows list
    S, W, diagonal, E, N). Horizontal couplings have magnitude kx * U(0.5, 1), vertical ones
    ky * U(0.5, 1); they are negative except for a fraction ``flip`` of positive ones, and a
    fraction ``one_way`` of them is zero (structurally nonsymmetric). Zero couplings are not
    stored. The diagonal is (1 + margin) times the row's absolute off-diagonal sum (1 where
    that sum is 0)."""
    n = nx * ny
    iy, ix = np.divmod(np.arange(n), nx)
    mag = np.stack([ky * r.uniform(0.5, 1.0, n), kx * r.uniform(0.5, 1.0, n),
                    np.zeros(n), kx * r.uniform(0.5, 1.0, n), ky * r.uniform(0.5, 1.0, n)], -1)
    sign = np.where(r.random((n, 5)) < flip, 1.0, -1.0)
    coef = mag * sign * (r.random((n, 5)) >= one_way)
    exists = np.stack([iy > 0, ix > 0, np.ones(n, bool), ix < nx - 1, iy < ny - 1], -1)
    coef = np.where(exists, coef, 0.0)
    s = np.abs(coef).sum(1)
    coef[:, 2] = np.where(s > 0, (1.0 + margin) * s, 1.0)
    keep = exists & ((coef != 0.0) | (np.arange(5) == 2))
    cols = (np.arange(n)[:, None] + np.array([-nx, -1, 0, 1, nx]))[keep].astype(np.int32)
    vals = coef[keep]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(keep.sum(1))
    return CSR(n, rowptr, cols, vals, {"grid": (nx, ny)})


# ---------------------------------------------------------------------------------------
# The analytic test problems of the paper's numerical section (Sec. 5): variable-coefficient
# operators a phi_xx + b phi_yy + alpha phi_x + beta phi_y on the unit square with Dirichlet
# data and source from a manufactured solution. Discretised here by second-order central
# differences on the vertex-centred n x n interior grid, h = 1/(n+1), unscaled (1/h^2).
# ---------------------------------------------------------------------------------------

def _sec5_stand_alone():
    pi = np.pi
    coef = (lambda x, y: np.exp(-x * (y + 2.0)) + 10.0,
            lambda x, y: np.exp(-2.0 * x + 2.0 * y) * np.cos(2 * pi * (2 * x + y / 2)) ** 2 + 3.0,
            lambda x, y: np.cos(pi * (x + y / 2)) * np.cos(2 * pi * x) + 4.0,
            lambda x, y: np.exp(2.0 * x - 2.0 * y))
    phi = lambda x, y: np.cos(pi * x) * np.cos(pi * y)
    d = {"x": lambda x, y: -pi * np.sin(pi * x) * np.cos(pi * y),
         "y": lambda x, y: -pi * np.cos(pi * x) * np.sin(pi * y),
         "xx": lambda x, y: -pi * pi * phi(x, y),
         "yy": lambda x, y: -pi * pi * phi(x, y)}
    return coef, phi, d


def _sec5_boundary_layers(eps):
    one = lambda x, y: np.ones(np.broadcast(x, y).shape)
    coef = (lambda x, y: -eps * one(x, y), lambda x, y: -eps * one(x, y), one, one)
    den = np.exp(-1.0 / eps) - 1.0
    phi = lambda x, y: (2 * np.exp(-1.0 / eps) - np.exp((x - 1) / eps) - np.exp((y - 1) / eps)) / den
    d = {"x": lambda x, y: -np.exp((x - 1) / eps) / eps / den + 0 * y,
         "y": lambda x, y: -np.exp((y - 1) / eps) / eps / den + 0 * x,
         "xx": lambda x, y: -np.exp((x - 1) / eps) / eps ** 2 / den + 0 * y,
         "yy": lambda x, y: -np.exp((y - 1) / eps) / eps ** 2 / den + 0 * x}
    return coef, phi, d


def _sec5_inner_layers(eps):
    one = lambda x, y: np.ones(np.broadcast(x, y).shape)
    coef = (lambda x, y: eps * one(x, y), lambda x, y: eps * one(x, y),
            lambda x, y: x + 0 * y, lambda x, y: y + 0 * x)
    phi = lambda x, y: np.exp(-(x + y - 1) ** 2 / eps)
    d1 = lambda x, y: -2 * (x + y - 1) / eps * phi(x, y)
    d2 = lambda x, y: (-2 / eps + 4 * (x + y - 1) ** 2 / eps ** 2) * phi(x, y)
    return coef, phi, {"x": d1, "y": d1, "xx": d2, "yy": d2}


def _sec5_stretched(p, eta, eps):
    u = lambda t: 1.0 + ((t - 0.5) ** 2 + eta) ** p / eps
    zero = lambda x, y: np.zeros(np.broadcast(x, y).shape)
    coef = (lambda x, y: u(x) + 0 * y, lambda x, y: u(y) + 0 * x, zero, zero)
    pi = np.pi
    phi = lambda x, y: np.cos(2 * pi * (x + y)) * np.sin(2 * pi * (x - y))
    d = {"x": lambda x, y: 2 * pi * np.cos(4 * pi * x) + 0 * y,
         "y": lambda x, y: -2 * pi * np.cos(4 * pi * y) + 0 * x,
         "xx": lambda x, y: -8 * pi * pi * np.sin(4 * pi * x) + 0 * y,
         "yy": lambda x, y: 8 * pi * pi * np.sin(4 * pi * y) + 0 * x}
    return coef, phi, d


def _sec5_mixed_derivative(eps):
    one = lambda x, y: np.ones(np.broadcast(x, y).shape)
    zero = lambda x, y: np.zeros(np.broadcast(x, y).shape)
    coef = (one, one, zero, zero, lambda x, y: (2.0 - eps) * one(x, y))
    phi = lambda x, y: 2 * x ** 3 * y ** 4
    d = {"x": lambda x, y: 6 * x ** 2 * y ** 4, "y": lambda x, y: 8 * x ** 3 * y ** 3,
         "xx": lambda x, y: 12 * x * y ** 4, "yy": lambda x, y: 24 * x ** 3 * y ** 2,
         "xy": lambda x, y: 24 * x ** 2 * y ** 3}
    return coef, phi, d


SEC5_PROBLEMS = {
    "mixed_derivative": lambda eps=0.01: _sec5_mixed_derivative(eps),
    "stand_alone": lambda: _sec5_stand_alone(),
    "boundary_layers": lambda eps=0.02: _sec5_boundary_layers(eps),
    "inner_layers": lambda eps=0.015: _sec5_inner_layers(eps),
    "stretched": lambda p=20, eta=0.5, eps=1e-6: _sec5_stretched(p, eta, eps),
}


def sec5_problem(name: str, n: int = 63, **params):
    """Operator, right-hand side and exact nodal solution of one Sec. 5 problem on an
    n x n interior grid. Rows list their stencil columns in ascending order (S, W, diagonal,
    E, N; with a mixed derivative term the 9-point stencil SW, S, SE, W, diagonal, E, NW, N,
    NE, phi_xy by the centred 4-point formula); zeros are kept, so the pattern is the full
    stencil. Boundary neighbours move to the right-hand side with the exact solution's
    values."""
    coef, phi, d = SEC5_PROBLEMS[name](**params)
    x, y, h = _grid_xy(n)
    a, bb, al, be = (f(x, y) for f in coef[:4])
    cxy = coef[4](x, y) if len(coef) > 4 else None
    g = a * d["xx"](x, y) + bb * d["yy"](x, y) + al * d["x"](x, y) + be * d["y"](x, y)
    # stencil offsets (dx, dy) and coefficients
    offs = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
    st = [bb / h ** 2 - be / (2 * h), a / h ** 2 - al / (2 * h), -2 * (a + bb) / h ** 2,
          a / h ** 2 + al / (2 * h), bb / h ** 2 + be / (2 * h)]
    if cxy is not None:
        g = g + cxy * d["xy"](x, y)
        q = cxy / (4 * h ** 2)
        offs = [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]
        st = [q, st[0], -q, st[1], st[2], st[3], -q, st[4], q]
    st = np.stack(st, axis=-1)
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    rhs = g.copy()
    exists = []
    for k, (dx, dy) in enumerate(offs):
        jx, jy = ix + dx, iy + dy
        inside = (jx >= 0) & (jx < n) & (jy >= 0) & (jy < n)
        bnd = ~inside
        rhs[bnd] -= st[..., k][bnd] * phi((jx[bnd] + 1) * h, (jy[bnd] + 1) * h)
        exists.append(inside)
    exists = np.stack(exists, -1).reshape(n * n, len(offs))
    idx = (iy * n + ix)[..., None] + np.array([dy * n + dx for dx, dy in offs])
    cols = idx.reshape(n * n, len(offs))[exists].astype(np.int32)
    vals = st.reshape(n * n, len(offs))[exists]
    rowptr = np.zeros(n * n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(exists.sum(1))
    A = CSR(n * n, rowptr, cols, vals, {"grid": (n, n), "h": h, "problem": name, **params})
    return A, rhs.reshape(-1), phi(x, y).reshape(-1)


def sec5_hierarchy(name: str, J: int = 6, coarsest: int = 1, **params):
    """Rediscretised operators of one Sec. 5 problem on nested grids 2^l - 1 (finest first,
    down to ``coarsest`` points per side), and the fine right-hand side."""
    levels = []
    lvl = J
    b = None
    while True:
        n = 2 ** lvl - 1
        A, rhs, _ = sec5_problem(name, n, **params)
        if b is None:
            b = rhs
        levels.append(A)
        if n <= coarsest:
            break
        lvl -= 1
    return levels, b
