"""Seeded Cartesian reservoir models for the single-phase pressure equation.

Cells are numbered x-fastest, ``idx = i + nx*(j + ny*k)``, with ``k = 0`` the
top layer.  Face transmissibilities use the two-point flux approximation named
in the paper's "Discrete equations" section: the half-transmissibility of cell
``c`` towards one of its faces is ``t = K_c |face area| / (half cell width)``
and the face value is ``m / (1/t_a + 1/t_b)`` with ``m`` the product of the
fault multipliers on that face.  Mobility is 1 throughout.

Layout handed to the solver (both the oracle and the GPU library):

* ``tx[i]`` is the transmissibility of the face between cell ``i`` and its
  ``+x`` neighbour (0 on the last column, next to an inactive cell, or where
  no face exists); ``ty``/``tz`` likewise.
* ``bc_cell/bc_trans/bc_value`` list Dirichlet faces and bottom-hole-pressure
  well connections: each adds ``bc_trans`` to the cell's diagonal and
  ``bc_trans*bc_value`` to its right-hand side.
* ``source`` is the injection rate per cell (``> 0`` injects).

This module does no solver arithmetic: no operator assembly, basis, coarse
operator or iteration lives here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components


@dataclass
class Problem:
    dims: tuple
    h: tuple
    active: np.ndarray
    tx: np.ndarray
    ty: np.ndarray
    tz: np.ndarray
    bc_cell: np.ndarray
    bc_trans: np.ndarray
    bc_value: np.ndarray
    source: np.ndarray
    perm: np.ndarray
    fault: np.ndarray  # uint8 [3, N]: 1 where the +d face of the cell lies on a fault
    name: str = ""
    wells: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        nx, ny, nz = self.dims
        return nx * ny * nz

    @property
    def n_active(self) -> int:
        return int(self.active.sum())

    def with_source(self, source=None, bc_value=None, bc_trans=None) -> "Problem":
        """Copy with a replaced source / well term (same grid, same faces)."""
        import copy

        p = copy.copy(self)
        if source is not None:
            p.source = np.ascontiguousarray(source, dtype=np.float64)
        if bc_value is not None:
            p.bc_value = np.ascontiguousarray(bc_value, dtype=np.float64)
        if bc_trans is not None:
            p.bc_trans = np.ascontiguousarray(bc_trans, dtype=np.float64)
        return p


def rng_for(cfg: int, realisation: int = 0) -> np.random.Generator:
    """PCG64 stream for workload ``cfg`` and realisation index."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(1624 + 1000 * cfg + realisation)))


def _shape3(dims):
    nx, ny, nz = dims
    return (nz, ny, nx)


def half_transmissibility(perm: np.ndarray, dims, h, axis: int) -> np.ndarray:
    """``K |face| / (h_axis / 2)`` for faces normal to ``axis`` (0=x, 1=y, 2=z)."""
    area = float(np.prod(h)) / h[axis]
    return perm * area / (0.5 * h[axis])


def face_transmissibility(perm, dims, h, active, mult=None):
    """Return ``(tx, ty, tz)``, each ``[N]``; see the module docstring."""
    shp = _shape3(dims)
    act = active.reshape(shp)
    out = []
    for axis in range(3):
        t = half_transmissibility(perm, dims, h, axis).reshape(shp)
        T = np.zeros(shp)
        ax = 2 - axis  # numpy axis of the (nz, ny, nx) array
        n = shp[ax]
        if n > 1:
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax] = slice(0, n - 1)
            hi[ax] = slice(1, n)
            lo, hi = tuple(lo), tuple(hi)
            ta, tb = t[lo], t[hi]
            both = act[lo] & act[hi]
            val = np.zeros_like(ta)
            val[both] = 1.0 / (1.0 / ta[both] + 1.0 / tb[both])
            T[lo] = val
        if mult is not None:
            T = T * mult[axis].reshape(shp)
        out.append(np.ascontiguousarray(T.reshape(-1)))
    return tuple(out)


def _cell_centres(dims, h):
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i + 0.5) * h[0]).reshape(-1), ((j + 0.5) * h[1]).reshape(-1), ((k + 0.5) * h[2]).reshape(-1)


def _dirichlet_x_faces(perm, dims, h, active, p_left=1.0, p_right=0.0):
    """Dirichlet faces on x = 0 (value ``p_left``) and x = Lx (value ``p_right``)."""
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz)
    i = idx % nx
    t = half_transmissibility(perm, dims, h, 0)
    cells, trans, vals = [], [], []
    for side, val in ((0, p_left), (nx - 1, p_right)):
        c = idx[(i == side) & active]
        cells.append(c)
        trans.append(t[c])
        vals.append(np.full(c.size, val))
    return (np.concatenate(cells).astype(np.int32), np.concatenate(trans), np.concatenate(vals))


def _prune_unanchored(active, tx, ty, tz, dims, anchored_cells):
    """Deactivate active components that touch no boundary or well connection."""
    nx, ny, nz = dims
    N = nx * ny * nz
    rows, cols = [], []
    for T, step in ((tx, 1), (ty, nx), (tz, nx * ny)):
        a = np.nonzero(T > 0)[0]
        rows.append(a)
        cols.append(a + step)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    G = coo_matrix((np.ones(r.size), (r, c)), shape=(N, N)).tocsr()
    _, lab = connected_components(G, directed=False)
    good = np.zeros(lab.max() + 1, dtype=bool)
    good[lab[anchored_cells]] = True
    return active & good[lab]


def make_homogeneous(dims, h=(1.0, 1.0, 1.0), K=1.0, p_left=1.0, p_right=0.0, name="homogeneous"):
    """Constant permeability box with Dirichlet ``x = 0`` / ``x = Lx`` faces."""
    N = int(np.prod(dims))
    perm = np.full(N, float(K))
    active = np.ones(N, dtype=bool)
    tx, ty, tz = face_transmissibility(perm, dims, h, active)
    bc = _dirichlet_x_faces(perm, dims, h, active, p_left, p_right)
    return Problem(tuple(dims), tuple(h), active, tx, ty, tz, *bc, np.zeros(N), perm,
                   np.zeros((3, N), np.uint8), name)


def make_lognormal_box(dims, rng, sigma=1.0, corr=None, h=(1.0, 1.0, 1.0), name="lognormal"):
    """``K = exp(sigma * z)``, ``z`` iid N(0,1) (optionally Gaussian-smoothed with
    per-axis std ``corr`` in cells, x/y/z order, and rescaled to unit variance);
    Dirichlet p=1 on x=0, p=0 on x=Lx, no flow elsewhere."""
    shp = _shape3(dims)
    z = rng.standard_normal(shp)
    if corr is not None:
        z = ndimage.gaussian_filter(z, sigma=(corr[2], corr[1], corr[0]), mode="reflect")
        z = (z - z.mean()) / z.std()
    perm = np.exp(sigma * z).reshape(-1)
    N = perm.size
    active = np.ones(N, dtype=bool)
    tx, ty, tz = face_transmissibility(perm, dims, h, active)
    bc = _dirichlet_x_faces(perm, dims, h, active)
    return Problem(tuple(dims), tuple(h), active, tx, ty, tz, *bc, np.zeros(N), perm,
                   np.zeros((3, N), np.uint8), name)


def make_config0(seed: int = 0):
    """60x60 unit cells, K = exp(N(0,1)) iid, p=1 left / p=0 right."""
    return make_lognormal_box((60, 60, 1), rng_for(0, seed), sigma=1.0, name=f"cfg0-s{seed}")


# --- layered lognormal + channel model with a five-spot well pattern --------

def _channel_perm(dims, rng, n_top):
    """Top ``n_top`` layers: smooth lognormal (sigma_lnK = 2, Gaussian filter
    std 4/8/1 cells in x/y/z).  Remaining layers: background 1 with six
    sinusoidal high-permeability (1000) channels per layer running along y."""
    nx, ny, nz = dims
    perm = np.ones((nz, ny, nx))
    if n_top > 0:
        z = rng.standard_normal((n_top, ny, nx))
        z = ndimage.gaussian_filter(z, sigma=(1.0, 8.0, 4.0), mode="reflect")
        z = (z - z.mean()) / z.std()
        perm[:n_top] = np.exp(2.0 * z)
    xc = np.arange(nx) + 0.5
    yc = np.arange(ny) + 0.5
    for k in range(n_top, nz):
        for _ in range(6):
            x0 = rng.uniform(0.0, nx)
            amp = rng.uniform(3.0, 10.0)
            lam = rng.uniform(50.0, 150.0)
            phi = rng.uniform(0.0, 2 * np.pi)
            width = int(rng.integers(2, 6))
            centre = x0 + amp * np.sin(2 * np.pi * yc / lam + phi)  # [ny]
            inside = np.abs(xc[None, :] - centre[:, None]) <= 0.5 * width
            perm[k][inside] = 1000.0
    return perm.reshape(-1)


def _five_spot(perm, dims, h, active, rate=1.0, rw=0.25):
    """Rate injector in the centre column (rate split evenly over its active
    cells) and four corner producers, each cell a bottom-hole-pressure
    connection to p=0 with Peaceman index 2 pi K dz / ln(r0/rw),
    r0 = 0.14 sqrt(dx^2 + dy^2)."""
    nx, ny, nz = dims
    dx, dy, dz = h
    N = nx * ny * nz
    col = lambda i, j: np.array([i + nx * (j + ny * k) for k in range(nz)], dtype=np.int64)
    inj = col(nx // 2, ny // 2)
    inj = inj[active[inj]]
    source = np.zeros(N)
    source[inj] = rate / max(inj.size, 1)
    r0 = 0.14 * np.sqrt(dx * dx + dy * dy)
    cells = []
    for (i, j) in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)):
        c = col(i, j)
        cells.append(c[active[c]])
    cells = np.concatenate(cells)
    wi = 2 * np.pi * perm[cells] * dz / np.log(r0 / rw)
    wells = {"injector": inj, "producers": cells}
    return source, cells.astype(np.int32), wi, np.zeros(cells.size), wells


def _well_cells(dims):
    nx, ny, nz = dims
    cols = [(nx // 2, ny // 2), (0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]
    return np.array([i + nx * (j + ny * k) for (i, j) in cols for k in range(nz)], dtype=np.int64)


def make_config1(dims=(60, 220, 85), h=(20.0, 10.0, 2.0), n_top=None, seed=0, name=None):
    """Layered model: smooth lognormal top, channelised bottom, five-spot wells.

    Full size is 60x220x85 (1,122,000 cells) with 35 lognormal layers; smaller
    ``dims`` keep the same recipe with ``n_top = round(35/85 * nz)``."""
    rng = rng_for(1, seed)
    nx, ny, nz = dims
    if n_top is None:
        n_top = int(round(35.0 * nz / 85.0))
    perm = _channel_perm(dims, rng, n_top)
    active = np.ones(nx * ny * nz, dtype=bool)
    tx, ty, tz = face_transmissibility(perm, dims, h, active)
    source, bc_cell, bc_trans, bc_value, wells = _five_spot(perm, dims, h, active)
    return Problem(tuple(dims), tuple(h), active, tx, ty, tz, bc_cell, bc_trans, bc_value, source,
                   perm, np.zeros((3, active.size), np.uint8), name or f"cfg1-{nx}x{ny}x{nz}-s{seed}", wells)


def _faults(dims, h, rng, n_faults=3):
    """Planar faults: a point uniform in the domain, normal (cos t, sin t, nz)
    normalised with t ~ U[0, pi), nz ~ U[-0.3, 0.3]; a face is cut when its two
    cell centres lie on different sides (sign(0) counts as +).  Each fault has
    one multiplier ~ U[0, 0.1]; multipliers of overlapping faults multiply."""
    nx, ny, nz = dims
    N = nx * ny * nz
    X, Y, Z = _cell_centres(dims, h)
    L = np.array([nx * h[0], ny * h[1], nz * h[2]])
    mult = np.ones((3, N))
    fault = np.zeros((3, N), np.uint8)
    for _ in range(n_faults):
        x0 = rng.uniform(0.0, 1.0, 3) * L
        th = rng.uniform(0.0, np.pi)
        n = np.array([np.cos(th), np.sin(th), rng.uniform(-0.3, 0.3)])
        n /= np.linalg.norm(n)
        m = rng.uniform(0.0, 0.1)
        side = (n[0] * (X - x0[0]) + n[1] * (Y - x0[1]) + n[2] * (Z - x0[2])) >= 0.0
        for axis, step, ncoord in ((0, 1, nx), (1, nx, ny), (2, nx * ny, nz)):
            coord = (np.arange(N) // step) % ncoord
            a = np.nonzero(coord < ncoord - 1)[0]
            cut = a[side[a] != side[a + step]]
            mult[axis, cut] *= m
            fault[axis, cut] = 1
    return mult, fault


def make_config2(dims=(60, 220, 85), h=(20.0, 10.0, 2.0), n_top=None, seed=0, p_inactive=0.05, name=None):
    """The layered five-spot model with three faults and iid inactive cells
    (probability 0.05, well columns kept active, components without a well or
    boundary connection removed)."""
    rng = rng_for(2, seed)
    nx, ny, nz = dims
    if n_top is None:
        n_top = int(round(35.0 * nz / 85.0))
    perm = _channel_perm(dims, rng, n_top)
    mult, fault = _faults(dims, h, rng)
    N = nx * ny * nz
    active = rng.uniform(size=N) >= p_inactive
    wc = _well_cells(dims)
    active[wc] = True
    tx, ty, tz = face_transmissibility(perm, dims, h, active, mult)
    active = _prune_unanchored(active, tx, ty, tz, dims, wc[active[wc]])
    tx, ty, tz = face_transmissibility(perm, dims, h, active, mult)
    fault = fault * np.stack([(tx > 0), (ty > 0), (tz > 0)]).astype(np.uint8)
    source, bc_cell, bc_trans, bc_value, wells = _five_spot(perm, dims, h, active)
    return Problem(tuple(dims), tuple(h), active, tx, ty, tz, bc_cell, bc_trans, bc_value, source,
                   perm, fault, name or f"cfg2-{nx}x{ny}x{nz}-s{seed}", wells)


def make_config3_member(member: int):
    """Ensemble member: nx, ny ~ U{32..128}, nz ~ U{8..16}; K = exp(2 z) with
    isotropic correlation length l ~ U[2, 16] cells (Gaussian filter std l/2);
    unit cells; p=1 left / p=0 right."""
    rng = rng_for(3, member)
    nx = int(rng.integers(32, 129))
    ny = int(rng.integers(32, 129))
    nz = int(rng.integers(8, 17))
    ell = rng.uniform(2.0, 16.0)
    s = ell / 2.0
    return make_lognormal_box((nx, ny, nz), rng, sigma=2.0, corr=(s, s, s), name=f"cfg3-m{member}")


def pressure_increment_pair(problem: Problem, rng: np.random.Generator):
    """Two synthetic pressure increments (newest first) with the structure the
    dynamic basis targets: a smooth global part plus sharp local changes
    around a random cell (a moved/rescaled well)."""
    nx, ny, nz = problem.dims
    X, Y, Z = _cell_centres(problem.dims, (1.0, 1.0, 1.0))
    out = []
    for _ in range(2):
        c = rng.uniform(0, 1, 3) * np.array([nx, ny, nz])
        r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        width = rng.uniform(2.0, 6.0)
        dp = np.exp(-r2 / (2 * width * width)) * rng.uniform(0.5, 2.0)
        dp += 1e-3 * rng.standard_normal(dp.size)
        dp[~problem.active] = 0.0
        out.append(dp)
    return out
