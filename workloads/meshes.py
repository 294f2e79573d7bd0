"""Seeded simplicial meshes standing in for the paper's meshes.

The paper's meshes exist only in its figures, so these generators produce
meshes of the same kind: Delaunay triangulations of jittered lattices on the
unit disk (Example 1), a graded L-shaped domain (Example 3), star-shaped
polygons, and the unit ball (Example 4).  Every vertex array is float64 and
row-major (N_v x d); every element array is int32 (N_e x (d+1)), 0-based and
positively oriented.  Vertices are numbered row by row (sorted by y, then x;
in 3D by z, y, x), which is the "natural" ordering the preconditioner uses.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import Delaunay, cKDTree


@dataclasses.dataclass
class Mesh:
    X: np.ndarray       # (nv, d) float64
    elems: np.ndarray   # (ne, d+1) int32
    name: str = ""

    @property
    def d(self) -> int:
        return int(self.X.shape[1])

    @property
    def nv(self) -> int:
        return int(self.X.shape[0])

    @property
    def ne(self) -> int:
        return int(self.elems.shape[0])


# ----------------------------------------------------------------------------
# helpers (geometry of the *generator*, not of the method)


def _signed_volumes(X, elems):
    d = X.shape[1]
    P = X[elems]                       # ne, d+1, d
    E = P[:, 1:, :] - P[:, :1, :]      # ne, d, d
    return np.linalg.det(E) / math.factorial(d)


def _orient_positive(X, elems):
    vol = _signed_volumes(X, elems)
    elems = elems.copy()
    neg = vol < 0
    elems[neg, 0], elems[neg, 1] = elems[neg, 1].copy(), elems[neg, 0].copy()
    return elems


def _natural_order(X, elems):
    """Renumber vertices row by row (last coordinate slowest)."""
    d = X.shape[1]
    keys = tuple(np.round(X[:, a], 12) for a in range(d))  # lexsort: last key primary
    order = np.lexsort(keys)
    inv = np.empty_like(order)
    inv[order] = np.arange(order.size)
    return X[order].copy(), inv[elems].astype(np.int32)


def _finish(X, elems, name, min_rel_vol=1e-10):
    X = np.ascontiguousarray(X, dtype=np.float64)
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    used = np.unique(elems)
    if used.size != X.shape[0]:
        remap = -np.ones(X.shape[0], dtype=np.int64)
        remap[used] = np.arange(used.size)
        X = X[used]
        elems = remap[elems]
    elems = _orient_positive(X, elems)
    vol = _signed_volumes(X, elems)
    if np.any(vol <= min_rel_vol * np.median(vol)):
        raise RuntimeError(f"{name}: degenerate element generated")
    X, elems = _natural_order(X, elems)
    return Mesh(X=np.ascontiguousarray(X), elems=np.ascontiguousarray(elems, dtype=np.int32), name=name)


def _hex_lattice(lo, hi, a, rng):
    """Hexagonal lattice of spacing a covering the box [lo, hi]^2 (random offset)."""
    off = rng.uniform(0, a, size=2)
    dy = a * math.sqrt(3) / 2
    ys = np.arange(lo[1] - a + off[1], hi[1] + a, dy)
    pts = []
    for r, y in enumerate(ys):
        xs = np.arange(lo[0] - a + off[0] + (0.5 * a if r % 2 else 0.0), hi[0] + a, a)
        pts.append(np.stack([xs, np.full_like(xs, y)], axis=1))
    return np.concatenate(pts, axis=0)


def _boundary_edges(elems):
    """Facets owned by exactly one element (2D: edges)."""
    e = np.concatenate([elems[:, [0, 1]], elems[:, [1, 2]], elems[:, [2, 0]]])
    e.sort(axis=1)
    uniq, cnt = np.unique(e, axis=0, return_counts=True)
    return uniq[cnt == 1]


def _check_polygon_mesh(X, elems, poly_area, name):
    area = _signed_volumes(X, elems).sum()
    if abs(area - poly_area) > 1e-9 * poly_area:
        raise RuntimeError(f"{name}: mesh area {area} != domain area {poly_area}")


# ----------------------------------------------------------------------------
# 2D generators


def disk_mesh(seed: int = 1001, n_boundary: int = 100, spacing: float = 0.058,
              jitter: float = 0.2) -> Mesh:
    """Unit disk: equispaced boundary points plus a jittered hexagonal lattice."""
    rng = np.random.default_rng(seed)
    t = 2 * np.pi * np.arange(n_boundary) / n_boundary
    bnd = np.stack([np.cos(t), np.sin(t)], axis=1)
    pts = _hex_lattice((-1, -1), (1, 1), spacing, rng)
    pts = pts + rng.uniform(-jitter * spacing, jitter * spacing, size=pts.shape)
    r = np.hypot(pts[:, 0], pts[:, 1])
    pts = pts[r < 1 - 0.5 * spacing]
    X = np.concatenate([bnd, pts])
    elems = Delaunay(X).simplices
    return _finish(X, elems, f"disk(seed={seed})")


def _polyline_points(corners, hfun):
    """Sample a closed polygon with local spacing hfun, keeping the corners."""
    out = []
    nc = len(corners)
    for c in range(nc):
        a = np.asarray(corners[c], dtype=np.float64)
        b = np.asarray(corners[(c + 1) % nc], dtype=np.float64)
        length = np.linalg.norm(b - a)
        # integrate 1/h along the segment to pick the number of points
        ts = np.linspace(0, 1, 2001)
        p = a[None, :] + ts[:, None] * (b - a)[None, :]
        dens = 1.0 / hfun(p)
        cum = np.concatenate([[0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(ts) * length)])
        m = max(1, int(round(cum[-1])))
        targets = np.linspace(0, cum[-1], m + 1)[:-1]
        tt = np.interp(targets, cum, ts)
        out.append(a[None, :] + tt[:, None] * (b - a)[None, :])
    return np.concatenate(out, axis=0)


def _dist_to_polyline(p, corners):
    d = np.full(p.shape[0], np.inf)
    nc = len(corners)
    for c in range(nc):
        a = np.asarray(corners[c], dtype=np.float64)
        b = np.asarray(corners[(c + 1) % nc], dtype=np.float64)
        ab = b - a
        t = np.clip(((p - a) @ ab) / (ab @ ab), 0, 1)
        q = a[None, :] + t[:, None] * ab[None, :]
        d = np.minimum(d, np.linalg.norm(p - q, axis=1))
    return d


def _graded_points(inside, hfun, box_lo, box_hi, hmin, hmax, rng, dist_fn, jitter=0.15):
    """Candidate interior points whose spacing follows hfun, then greedy thinning."""
    cands = []
    h = hmin
    while True:
        lat = _hex_lattice(box_lo, box_hi, h, rng)
        lat = lat + rng.uniform(-jitter * h, jitter * h, size=lat.shape)
        hl = hfun(lat)
        last = h * 2 > hmax
        keep = (hl >= h) & ((hl < 2 * h) | last) & inside(lat)
        lat = lat[keep]
        hl = hl[keep]
        keep = dist_fn(lat) >= 0.6 * hl
        cands.append(lat[keep])
        if last:
            break
        h *= 2
    P = np.concatenate(cands)
    hl = hfun(P)
    order = np.argsort(hl, kind="stable")
    P = P[order]
    hl = hl[order]
    tree = cKDTree(P)
    nbrs = tree.query_ball_point(P, 0.7 * hl)
    accepted = np.zeros(P.shape[0], dtype=bool)
    for i in range(P.shape[0]):
        ok = True
        for j in nbrs[i]:
            if accepted[j]:
                ok = False
                break
        if ok:
            accepted[i] = True
    return P[accepted]


def lshape_mesh(seed: int = 1002, hmin: float = 0.006, hmax: float = 0.0075,
                r0: float = 0.5) -> Mesh:
    """L-shaped domain [-1,1]^2 minus [0,1]^2, graded toward the reentrant corner.

    Local spacing grows from hmin at the corner (0,0) to hmax at distance r0
    and beyond (a square-root profile).  The defaults give about 65k vertices
    with a minimum element height just above 2/1024, the spacing of a
    1024 x 1024 overlay grid on [-1,1]^2.
    """
    rng = np.random.default_rng(seed)
    corners = [(-1, -1), (1, -1), (1, 0), (0, 0), (0, 1), (-1, 1)]

    def hfun(p):
        r = np.hypot(p[:, 0], p[:, 1])
        return np.minimum(hmax, hmin + (hmax - hmin) * np.sqrt(np.minimum(r, r0) / r0))

    def inside(p):
        return (np.abs(p[:, 0]) < 1) & (np.abs(p[:, 1]) < 1) & ~((p[:, 0] > 0) & (p[:, 1] > 0))

    bnd = _polyline_points(corners, hfun)
    pts = _graded_points(inside, hfun, (-1, -1), (1, 1), hmin, hmax, rng,
                         lambda q: _dist_to_polyline(q, corners))
    X = np.concatenate([bnd, pts])
    tri = Delaunay(X).simplices
    cen = X[tri].mean(axis=1)
    tri = tri[~((cen[:, 0] > 0) & (cen[:, 1] > 0))]
    _check_polygon_mesh(X, tri, 3.0, "lshape")
    return _finish(X, tri, f"lshape(seed={seed})")


def star_radius_fn(seed: int):
    """r(theta) = 1 + 0.3 * sum_{m=1..5} a_m cos(m theta + phi_m), min r >= 0.3."""
    rng = np.random.default_rng(seed)
    while True:
        a = rng.uniform(0, 0.4, size=5)
        phi = rng.uniform(0, 2 * np.pi, size=5)
        m = np.arange(1, 6)

        def r(theta, a=a, phi=phi):
            theta = np.asarray(theta, dtype=np.float64)
            return 1 + 0.3 * np.sum(a[:, None] * np.cos(m[:, None] * theta[None, :] + phi[:, None]), axis=0)

        tt = np.linspace(0, 2 * np.pi, 4096, endpoint=False)
        if r(tt).min() >= 0.3:
            return r


def star_mesh(seed: int, nv_target: int) -> Mesh:
    """Quasi-uniform mesh of a seeded random star-shaped polygon."""
    rfun = star_radius_fn(seed)
    rng = np.random.default_rng(seed + 7)
    tt = np.linspace(0, 2 * np.pi, 20000, endpoint=False)
    rr = rfun(tt)
    area = 0.5 * np.mean(rr ** 2) * 2 * np.pi
    h = math.sqrt(area / nv_target * 2 / math.sqrt(3))
    # boundary: equal arc length sampling of the dense curve
    dense = np.stack([rr * np.cos(tt), rr * np.sin(tt)], axis=1)
    seg = np.linalg.norm(np.roll(dense, -1, axis=0) - dense, axis=1)
    cum = np.concatenate([[0], np.cumsum(seg)])
    perim = cum[-1]
    m = max(16, int(round(perim / h)))
    targets = np.linspace(0, perim, m, endpoint=False)
    tb = np.interp(targets, cum, np.concatenate([tt, [2 * np.pi]]))
    rb = rfun(tb)
    bnd = np.stack([rb * np.cos(tb), rb * np.sin(tb)], axis=1)
    rmax = rr.max()
    pts = _hex_lattice((-rmax, -rmax), (rmax, rmax), h, rng)
    pts = pts + rng.uniform(-0.15 * h, 0.15 * h, size=pts.shape)
    th = np.arctan2(pts[:, 1], pts[:, 0])
    inside = np.hypot(pts[:, 0], pts[:, 1]) < rfun(th)
    pts = pts[inside]
    tree = cKDTree(dense)
    dist, _ = tree.query(pts)
    pts = pts[dist >= 0.6 * h]
    X = np.concatenate([bnd, pts])
    tri = Delaunay(X).simplices
    cen = X[tri].mean(axis=1)
    thc = np.arctan2(cen[:, 1], cen[:, 0])
    tri = tri[np.hypot(cen[:, 0], cen[:, 1]) < rfun(thc)]
    # polygon area by the shoelace formula
    pa = 0.5 * np.sum(bnd[:, 0] * np.roll(bnd[:, 1], -1) - np.roll(bnd[:, 0], -1) * bnd[:, 1])
    _check_polygon_mesh(X, tri, pa, "star")
    return _finish(X, tri, f"star(seed={seed},nv~{nv_target})")


def structured_box_mesh(grid_lo, h, nx, ny, flip=False) -> Mesh:
    """Grid-coincident triangulation: vertices at lo + (i h, j h), each square split in two.

    With the mesh vertices placed exactly on overlay-grid nodes (same lo and
    h), P1 interpolation to the grid reduces to a selection.
    """
    lo = np.asarray(grid_lo, dtype=np.float64)
    i = np.arange(nx + 1, dtype=np.float64)
    j = np.arange(ny + 1, dtype=np.float64)
    xs = lo[0] + i * np.float64(h)
    ys = lo[1] + j * np.float64(h)
    XX, YY = np.meshgrid(xs, ys, indexing="xy")
    X = np.stack([XX.ravel(), YY.ravel()], axis=1)
    tris = []
    for b in range(ny):
        for a in range(nx):
            v00 = b * (nx + 1) + a
            v10 = v00 + 1
            v01 = v00 + nx + 1
            v11 = v01 + 1
            if (a + b + (1 if flip else 0)) % 2 == 0:
                tris += [(v00, v10, v11), (v00, v11, v01)]
            else:
                tris += [(v00, v10, v01), (v10, v11, v01)]
    return _finish(X, np.array(tris), f"structured({nx}x{ny})")


def structured_box_mesh_3d(grid_lo, h, nx, ny, nz) -> Mesh:
    """Grid-coincident tetrahedral mesh: each cube split into 6 tetrahedra (Kuhn)."""
    lo = np.asarray(grid_lo, dtype=np.float64)
    xs = lo[0] + np.arange(nx + 1, dtype=np.float64) * np.float64(h)
    ys = lo[1] + np.arange(ny + 1, dtype=np.float64) * np.float64(h)
    zs = lo[2] + np.arange(nz + 1, dtype=np.float64) * np.float64(h)
    ZZ, YY, XX = np.meshgrid(zs, ys, xs, indexing="ij")
    X = np.stack([XX.ravel(), YY.ravel(), ZZ.ravel()], axis=1)

    def vid(a, b, c):
        return (c * (ny + 1) + b) * (nx + 1) + a

    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for c in range(nz):
        for b in range(ny):
            for a in range(nx):
                for p in perms:
                    cur = [a, b, c]
                    vs = [vid(*cur)]
                    for ax in p:
                        cur[ax] += 1
                        vs.append(vid(*cur))
                    tets.append(vs)
    return _finish(X, np.array(tets), f"structured3d({nx}x{ny}x{nz})")


# ----------------------------------------------------------------------------
# 3D generator


def _fibonacci_sphere(n):
    k = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * k / n)
    theta = np.pi * (1 + 5 ** 0.5) * k
    return np.stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)], axis=1)


def ball_mesh(seed: int = 1003, spacing: float = 0.0285, jitter: float = 0.15) -> Mesh:
    """Unit ball: jittered cubic lattice plus Fibonacci-sphere surface points.

    The default spacing gives about 200k vertices.  Surface points are pulled
    inward by a tiny random amount so that no four of them are exactly
    cospherical with the boundary sphere (the mesh approximately fits the ball).
    """
    rng = np.random.default_rng(seed)
    g = np.arange(-1 - spacing, 1 + spacing, spacing) + rng.uniform(0, spacing)
    Z, Y, Xg = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([Xg.ravel(), Y.ravel(), Z.ravel()], axis=1)
    pts = pts + rng.uniform(-jitter * spacing, jitter * spacing, size=pts.shape)
    pts = pts[np.linalg.norm(pts, axis=1) < 1 - 0.6 * spacing]
    nsurf = int(round(4 * np.pi / (spacing ** 2 * math.sqrt(3) / 2)))
    surf = _fibonacci_sphere(nsurf)
    surf = surf * (1 - rng.uniform(0, 1e-3 * spacing, size=(nsurf, 1)))
    X = np.concatenate([surf, pts])
    tets = Delaunay(X).simplices
    vol = np.abs(_signed_volumes(X, tets))
    tets = tets[vol > 1e-9 * spacing ** 3]
    return _finish(X, tets, f"ball(seed={seed})", min_rel_vol=1e-12)


def interval_mesh(n: int, seed: int | None = None, jitter: float = 0.0, a: float = -1.0, b: float = 1.0) -> Mesh:
    """The interval (a, b) in n elements: equispaced vertices, interior ones moved by up to jitter times the
    spacing (seeded); X is (n+1) x 1, increasing, elements (e, e+1)."""
    x = np.linspace(a, b, n + 1)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        x[1:-1] += rng.uniform(-jitter, jitter, n - 1) * (b - a) / n
    elems = np.stack([np.arange(n), np.arange(1, n + 1)], axis=1).astype(np.int32)
    return Mesh(x[:, None], elems, f"interval(n={n}, seed={seed})")
