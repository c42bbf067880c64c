"""Seeded synthetic triangulations.

This module only builds point sets and triangle lists (plus the node-pair
segments that tag open boundaries).  It holds none of the finite-volume
arithmetic: no areas, normals, edge tables or fluxes.  Both the FP64 oracle and
the HIP library derive their own geometry from what is returned here.

All generators return ``(xy, tri, sides)`` where ``xy`` is ``(V, 2)`` float64,
``tri`` is ``(N, 3)`` int32 with counter-clockwise vertex order, and ``sides``
maps a side name (``"x0"``, ``"x1"``, ``"y0"``, ``"y1"``) to the node ids lying
on that side of the rectangle, sorted along it.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import Delaunay


def _ccw(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Reorder each triangle counter-clockwise (generators promise CCW)."""
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    cross = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    tri = tri.copy()
    flip = cross < 0
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri.astype(np.int32)


def _sides(xy: np.ndarray, lx: float, ly: float, x0: float = 0.0, y0: float = 0.0):
    tol = 1e-9 * max(lx, ly)
    out = {}
    for name, mask, key in (
        ("x0", np.abs(xy[:, 0] - x0) <= tol, 1),
        ("x1", np.abs(xy[:, 0] - (x0 + lx)) <= tol, 1),
        ("y0", np.abs(xy[:, 1] - y0) <= tol, 0),
        ("y1", np.abs(xy[:, 1] - (y0 + ly)) <= tol, 0),
    ):
        ids = np.nonzero(mask)[0]
        out[name] = ids[np.argsort(xy[ids, key], kind="stable")].astype(np.int32)
    return out


def structured_right(lx: float, ly: float, d: float):
    """Rectangle [0,lx]x[0,ly] of d-sized squares, each cut along its
    (x0,y0)->(x0+d,y0+d) diagonal into two right triangles."""
    nx, ny = int(round(lx / d)), int(round(ly / d))
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xy = np.c_[X.ravel(), Y.ravel()]
    vid = np.arange((nx + 1) * (ny + 1)).reshape(ny + 1, nx + 1)
    v00 = vid[:-1, :-1].ravel()
    v10 = vid[:-1, 1:].ravel()
    v11 = vid[1:, 1:].ravel()
    v01 = vid[1:, :-1].ravel()
    t1 = np.c_[v00, v10, v11]
    t2 = np.c_[v00, v11, v01]
    tri = np.empty((2 * len(v00), 3), dtype=np.int32)
    tri[0::2] = t1
    tri[1::2] = t2
    return xy, tri, _sides(xy, lx, ly)


def _boundary_points(lx: float, ly: float, spacing: float) -> np.ndarray:
    nx = max(1, int(np.ceil(lx / spacing)))
    ny = max(1, int(np.ceil(ly / spacing)))
    bx = np.linspace(0.0, lx, nx + 1)
    by = np.linspace(0.0, ly, ny + 1)[1:-1]
    pts = [np.c_[bx, np.zeros_like(bx)], np.c_[bx, np.full_like(bx, ly)],
           np.c_[np.zeros_like(by), by], np.c_[np.full_like(by, lx), by]]
    return np.concatenate(pts)


def poisson_disk(lx: float, ly: float, r: float, rng: np.random.Generator,
                 rounds: int = 12) -> np.ndarray:
    """Seeded random points in [0,lx]x[0,ly] no two closer than ``r``.

    Boundary points sit on the four sides at spacing <= r.  Interior points
    are dart-thrown on a background grid of cell size r/sqrt(2) (at most one
    point per cell); cells are visited in nine interleaved phases so that
    darts of one phase can never conflict with each other, which lets a whole
    phase be tested at once.  After ``rounds`` sweeps the set is close to
    maximal, which is what keeps Delaunay angles large.
    """
    s = r / np.sqrt(2.0)
    gx, gy = int(np.ceil(lx / s)), int(np.ceil(ly / s))
    grid = np.full((gy + 4, gx + 4), -1, dtype=np.int64)  # 2-cell pad
    bpts = _boundary_points(lx, ly, r)
    # two boundary points can share a grid cell (the grid keeps one of them);
    # darts near the sides are therefore also tested against every boundary
    # point explicitly below
    ci = np.minimum((bpts[:, 0] / s).astype(np.int64), gx - 1) + 2
    cj = np.minimum((bpts[:, 1] / s).astype(np.int64), gy - 1) + 2
    grid[cj, ci] = np.arange(len(bpts))
    allx = bpts[:, 0].copy()
    ally = bpts[:, 1].copy()
    offs = [(di, dj) for dj in range(-2, 3) for di in range(-2, 3) if not (abs(di) == 2 and abs(dj) == 2)]
    II, JJ = np.meshgrid(np.arange(gx), np.arange(gy), indexing="xy")
    II = II.ravel()
    JJ = JJ.ravel()
    band = 0.8 * r
    for _ in range(rounds):
        added_any = False
        for ph in range(9):
            a, b = ph % 3, ph // 3
            m = (II % 3 == a) & (JJ % 3 == b)
            ii, jj = II[m], JJ[m]
            empty = grid[jj + 2, ii + 2] < 0
            ii, jj = ii[empty], jj[empty]
            if len(ii) == 0:
                continue
            x = (ii + rng.random(len(ii))) * s
            y = (jj + rng.random(len(jj))) * s
            ok = (x < lx) & (y < ly) & (x > band) & (y > band) & (x < lx - band) & (y < ly - band)
            for di, dj in offs:
                nb = grid[jj + 2 + dj, ii + 2 + di]
                has = nb >= 0
                d2 = np.full(len(ii), np.inf)
                d2[has] = (allx[nb[has]] - x[has]) ** 2 + (ally[nb[has]] - y[has]) ** 2
                ok &= d2 >= r * r
            # boundary points can be missed by the grid when two share a cell;
            # test the ones near the sides against all boundary points directly
            near = ok & ((x < 2 * r) | (y < 2 * r) | (x > lx - 2 * r) | (y > ly - 2 * r))
            if near.any():
                idx = np.nonzero(near)[0]
                d2b = ((x[idx, None] - bpts[None, :, 0]) ** 2 + (y[idx, None] - bpts[None, :, 1]) ** 2).min(axis=1)
                ok[idx[d2b < r * r]] = False
            if ok.any():
                added_any = True
                n0 = len(allx)
                newx, newy = x[ok], y[ok]
                allx = np.concatenate([allx, newx])
                ally = np.concatenate([ally, newy])
                grid[jj[ok] + 2, ii[ok] + 2] = n0 + np.arange(len(newx))
        if not added_any:
            break
    return np.c_[allx, ally]


def delaunay_rect(xy: np.ndarray, lx: float, ly: float):
    tri = Delaunay(xy).simplices.astype(np.int32)
    tri = _ccw(xy, tri)
    return xy, tri, _sides(xy, lx, ly)


def _fill_gaps(xy: np.ndarray, lx: float, ly: float, r: float, max_iter: int = 20) -> np.ndarray:
    """Insert the circumcentre of every Delaunay triangle whose circumradius
    exceeds ``r``.  Such a circle is empty, so its centre is at least ``r``
    from every point and the disk property survives; centres that would sit
    within ``r`` of each other are thinned greedily, largest circle first."""
    band = 0.8 * r
    for _ in range(max_iter):
        tri = Delaunay(xy).simplices
        a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
        d = 2 * (a[:, 0] * (b[:, 1] - c[:, 1]) + b[:, 0] * (c[:, 1] - a[:, 1]) + c[:, 0] * (a[:, 1] - b[:, 1]))
        a2, b2, c2 = (a * a).sum(1), (b * b).sum(1), (c * c).sum(1)
        ux = (a2 * (b[:, 1] - c[:, 1]) + b2 * (c[:, 1] - a[:, 1]) + c2 * (a[:, 1] - b[:, 1])) / d
        uy = (a2 * (c[:, 0] - b[:, 0]) + b2 * (a[:, 0] - c[:, 0]) + c2 * (b[:, 0] - a[:, 0])) / d
        R = np.sqrt((a[:, 0] - ux) ** 2 + (a[:, 1] - uy) ** 2)
        m = (R > r) & (ux > band) & (uy > band) & (ux < lx - band) & (uy < ly - band)
        if not m.any():
            break
        idx = np.nonzero(m)[0]
        idx = idx[np.argsort(-R[idx], kind="stable")]
        cand = np.c_[ux[idx], uy[idx]]
        keep = []
        cells = {}
        for k, (px, py) in enumerate(cand):
            ci, cj = int(px // r), int(py // r)
            ok = True
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    for qx, qy in cells.get((ci + di, cj + dj), ()):
                        if (qx - px) ** 2 + (qy - py) ** 2 < r * r:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                cells.setdefault((ci, cj), []).append((px, py))
                keep.append(k)
        if not keep:
            break
        xy = np.concatenate([xy, cand[keep]])
    return xy


def poisson_delaunay(lx: float, ly: float, n_target: int, rng: np.random.Generator):
    """Delaunay triangulation of a Poisson-disk point set with about
    ``n_target`` triangles.  A maximal disk sampling has every empty circle of
    radius below r and every edge at least r long, so no angle is under 30
    degrees; the near-maximal sampling here is checked to stay above 28."""
    # maximal Poisson-disk sets hold about 0.70 points per r^2 (measured on
    # this sampler); a planar triangulation has about 2 triangles per point
    r = np.sqrt(0.70 * lx * ly / (0.5 * n_target))
    xy = poisson_disk(lx, ly, r, rng)
    xy = _fill_gaps(xy, lx, ly, r)
    return delaunay_rect(xy, lx, ly)


def jittered_lattice(lx: float, ly: float, n_nodes: int, rng: np.random.Generator,
                     jitter: float = 0.25):
    """About ``n_nodes`` lattice points jittered by +-``jitter`` of the spacing
    (boundary points only slide along their side), then Delaunay."""
    h = np.sqrt(lx * ly / n_nodes)
    nx = max(2, int(round(lx / h)))
    ny = max(2, int(round(ly / h)))
    hx, hy = lx / nx, ly / ny
    X, Y = np.meshgrid(np.arange(nx + 1) * hx, np.arange(ny + 1) * hy, indexing="xy")
    xy = np.c_[X.ravel(), Y.ravel()]
    i = np.tile(np.arange(nx + 1), ny + 1)
    j = np.repeat(np.arange(ny + 1), nx + 1)
    jx = (rng.random(len(xy)) - 0.5) * 2 * jitter * hx
    jy = (rng.random(len(xy)) - 0.5) * 2 * jitter * hy
    jx[(i == 0) | (i == nx)] = 0.0
    jy[(j == 0) | (j == ny)] = 0.0
    # corners stay put; boundary nodes move only along their side
    xy[:, 0] += jx
    xy[:, 1] += jy
    return delaunay_rect(xy, lx, ly)


def min_angle_deg(xy: np.ndarray, tri: np.ndarray) -> float:
    """Smallest interior angle of the triangulation, for generator checks."""
    p = xy[tri]
    ang = []
    for k in range(3):
        a = p[:, (k + 1) % 3] - p[:, k]
        b = p[:, (k + 2) % 3] - p[:, k]
        cosv = (a * b).sum(1) / np.sqrt((a * a).sum(1) * (b * b).sum(1))
        ang.append(np.degrees(np.arccos(np.clip(cosv, -1, 1))))
    return float(np.min(ang))


def segments_on_side(xy: np.ndarray, side_ids: np.ndarray, lo: float, hi: float, axis: int):
    """Consecutive node pairs along one sorted side whose both ends lie within
    [lo, hi] along ``axis``.  On a triangulation of the rectangle consecutive
    side nodes are joined by a boundary edge."""
    c = xy[side_ids, axis]
    sel = []
    for a, b, ca, cb in zip(side_ids[:-1], side_ids[1:], c[:-1], c[1:]):
        if ca >= lo - 1e-9 and cb <= hi + 1e-9:
            sel.append((a, b))
    return np.asarray(sel, dtype=np.int32).reshape(-1, 2)
