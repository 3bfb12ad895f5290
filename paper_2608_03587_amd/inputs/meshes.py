"""Seeded synthetic triangular meshes of the transverse plane.

These generators produce the *inputs* of the method: vertex coordinates and
triangle connectivity.  They hold no discrete-exterior-calculus arithmetic
(no incidence matrices, Hodge stars or operators); both the CPU oracle and
the GPU library consume their output independently.

The paper meshes circular fibre cross-sections with an unnamed mesh tool and
states that triangles come out consistently oriented (Results, "DEC
computational framework").  No mesher is available here, so meshes are built
from NumPy point sets triangulated with ``scipy.spatial.Delaunay``:

* interior points on a jittered hexagonal lattice (near-equilateral
  triangles),
* circles that must conform (the domain boundary, a core-cladding interface,
  photonic-crystal-fibre holes) carry points placed exactly on the circle,
  with lattice points kept at least ``0.75 h`` away from them,
* graded meshes use concentric rings whose spacing follows ``h(r)``.

Every mesh is checked for a minimum interior angle and re-seeded on failure.
Triangles are returned in Qhull's order and orientation; orienting them is
the consumer's job.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import Delaunay

__all__ = [
    "Mesh",
    "min_angle_deg",
    "disk_mesh",
    "graded_core_disk_mesh",
    "pcf_mesh",
    "strip_mesh",
    "regular_grid_mesh",
    "hex_patch_mesh",
    "random_delaunay_mesh",
    "wheel_disk_mesh",
    "jittered_lattice_mesh",
]


@dataclass
class Mesh:
    """Vertex coordinates ``xy`` (float64 [N,2]) and triangles ``tri`` (int32 [T,3])."""

    xy: np.ndarray
    tri: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_vert(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    @property
    def r(self) -> np.ndarray:
        return np.hypot(self.xy[:, 0], self.xy[:, 1])


def min_angle_deg(xy: np.ndarray, tri: np.ndarray) -> float:
    """Smallest interior angle over all triangles, in degrees (mesh-quality check)."""
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]

    def angle(p, q, r):
        u = q - p
        v = r - p
        cosang = (u * v).sum(1) / (np.linalg.norm(u, axis=1) * np.linalg.norm(v, axis=1))
        return np.degrees(np.arccos(np.clip(cosang, -1.0, 1.0)))

    return float(np.min(np.minimum(np.minimum(angle(a, b, c), angle(b, c, a)), angle(c, a, b))))


def _hex_lattice(xmin, xmax, ymin, ymax, h):
    dy = h * math.sqrt(3.0) / 2.0
    j0 = int(math.floor(ymin / dy)) - 1
    j1 = int(math.ceil(ymax / dy)) + 1
    i0 = int(math.floor(xmin / h)) - 1
    i1 = int(math.ceil(xmax / h)) + 1
    jj = np.arange(j0, j1 + 1)
    ii = np.arange(i0, i1 + 1)
    X = ii[None, :] * h + 0.5 * h * (jj[:, None] & 1)
    Y = np.broadcast_to(jj[:, None] * dy, X.shape)
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def _ring(radius, n, rng, centre=(0.0, 0.0), angle_jitter=0.0, phase=None):
    n = max(int(n), 3)
    if phase is None:
        phase = rng.uniform(0.0, 2.0 * math.pi / n)
    th = phase + 2.0 * math.pi * np.arange(n) / n
    if angle_jitter > 0.0:
        th = th + rng.uniform(-angle_jitter, angle_jitter, n) * (2.0 * math.pi / n)
    return np.stack([centre[0] + radius * np.cos(th), centre[1] + radius * np.sin(th)], axis=1)


def _triangulate(pts: np.ndarray) -> np.ndarray:
    d = Delaunay(pts)
    return np.ascontiguousarray(d.simplices.astype(np.int32))


def _finish(pts, meta, min_angle):
    tri = _triangulate(pts)
    # drop vertices Qhull left unreferenced (coincident points); none expected
    used = np.zeros(len(pts), bool)
    used[tri.ravel()] = True
    if not used.all():
        remap = -np.ones(len(pts), np.int64)
        remap[used] = np.arange(used.sum())
        pts = pts[used]
        tri = remap[tri].astype(np.int32)
    ang = min_angle_deg(pts, tri)
    meta = dict(meta, min_angle_deg=ang)
    return Mesh(np.ascontiguousarray(pts, dtype=np.float64), tri, meta), ang >= min_angle


def _retry(builder, seed, min_angle, tries=8):
    last = None
    for k in range(tries):
        mesh, ok = builder(np.random.default_rng(seed + 7919 * k))
        mesh.meta["seed"] = seed
        mesh.meta["attempt"] = k
        if ok:
            return mesh
        last = mesh
    raise RuntimeError(
        f"mesh generator could not reach min angle {min_angle} deg (best {last.meta['min_angle_deg']:.2f})"
    )


def disk_mesh(R: float, h: float, seed: int, jitter: float = 0.05, min_angle: float = 25.0) -> Mesh:
    """Quasi-uniform disk of radius ``R``: jittered hex lattice plus an exact boundary ring."""

    def build(rng):
        p = _hex_lattice(-R, R, -R, R, h)
        p = p + rng.uniform(-jitter * h, jitter * h, p.shape)
        p = p[np.hypot(p[:, 0], p[:, 1]) <= R - 0.75 * h]
        ring = _ring(R, round(2 * math.pi * R / h), rng)
        return _finish(np.concatenate([p, ring]), {"kind": "disk", "R": R, "h": h}, min_angle)

    return _retry(build, seed, min_angle)


def _graded_h(r, r_core, h_core, h_max, R_grade, p):
    s = np.clip((r - r_core) / (R_grade - r_core), 0.0, None)
    return np.where(r <= r_core, h_core, np.minimum(h_max, h_core + (h_max - h_core) * s ** p))


def _ring_radii(r_core, R, h_core, h_max, p):
    """Concentric ring radii from ``r_core`` to ``R`` spaced by ``(sqrt3/2) h(r)``."""
    radii = [r_core]
    while radii[-1] < R:
        r = radii[-1]
        hr = float(_graded_h(r, r_core, h_core, h_max, R, p))
        hm = float(_graded_h(r + 0.433 * hr, r_core, h_core, h_max, R, p))
        radii.append(r + math.sqrt(3.0) / 2.0 * hm)
    radii = np.array(radii)
    # stretch so the last ring lands exactly on R
    radii = r_core + (radii - r_core) * (R - r_core) / (radii[-1] - r_core)
    return radii


def _graded_count(r_core, R, h_core, h_max, p):
    radii = _ring_radii(r_core, R, h_core, h_max, p)
    hs = _graded_h(radii, r_core, h_core, h_max, R, p)
    n_rings = np.maximum(3, np.round(2 * math.pi * radii / hs)).sum()
    n_core = math.pi * r_core**2 * 2.0 / (math.sqrt(3.0) * h_core**2)
    return n_rings + n_core


def graded_core_disk_mesh(
    R: float = 40.0,
    r_core: float = 5.0,
    h_core: float = 0.05,
    h_max: float = 0.4,
    target_vertices: int = 250_000,
    seed: int = 21,
    jitter: float = 0.05,
    min_angle: float = 25.0,
) -> Mesh:
    """Disk with a uniformly fine core and rings graded outward.

    Inside ``r <= r_core`` a hex lattice of spacing ``h_core``; an exact ring on
    ``r = r_core`` makes the core-cladding interface conform; outside, rings
    with spacing ``h(r) = min(h_max, h_core + (h_max-h_core) ((r-r_core)/(R-r_core))^p)``
    up to an exact ring on ``R``.  The exponent ``p`` is chosen by bisection so
    that the vertex count is close to ``target_vertices``.
    """
    lo, hi = 0.3, 6.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if _graded_count(r_core, R, h_core, h_max, mid) < target_vertices:
            lo = mid
        else:
            hi = mid
    p = 0.5 * (lo + hi)
    radii = _ring_radii(r_core, R, h_core, h_max, p)
    hs = _graded_h(radii, r_core, h_core, h_max, R, p)

    def build(rng):
        core = _hex_lattice(-r_core, r_core, -r_core, r_core, h_core)
        core = core + rng.uniform(-jitter * h_core, jitter * h_core, core.shape)
        core = core[np.hypot(core[:, 0], core[:, 1]) <= r_core - 0.75 * h_core]
        parts = [core]
        for k, (rk, hk) in enumerate(zip(radii, hs)):
            n = round(2 * math.pi * rk / hk)
            exact = k == 0 or k == len(radii) - 1
            ring = _ring(rk, n, rng, angle_jitter=0.0 if exact else jitter)
            if not exact:
                rr = rk + rng.uniform(-jitter * hk, jitter * hk, len(ring))
                ang = np.arctan2(ring[:, 1], ring[:, 0])
                ring = np.stack([rr * np.cos(ang), rr * np.sin(ang)], axis=1)
            parts.append(ring)
        meta = {"kind": "graded_core_disk", "R": R, "r_core": r_core, "h_core": h_core, "h_max": h_max, "p": p}
        return _finish(np.concatenate(parts), meta, min_angle)

    return _retry(build, seed, min_angle)


def pcf_hole_centres(pitch: float = 2.0, n_rings: int = 4) -> np.ndarray:
    """Centres of a hexagonal lattice of air holes with the central one removed."""
    cs = []
    for a in range(-n_rings, n_rings + 1):
        for b in range(-n_rings, n_rings + 1):
            if abs(a) > n_rings or abs(b) > n_rings or abs(a + b) > n_rings:
                continue
            if a == 0 and b == 0:
                continue
            cs.append((pitch * (a + 0.5 * b), pitch * (math.sqrt(3.0) / 2.0) * b))
    return np.array(cs, dtype=np.float64)


def pcf_mesh(
    h: float,
    hole_radius: float,
    seed: int,
    R: float = 12.0,
    pitch: float = 2.0,
    n_rings: int = 4,
    jitter: float = 0.05,
    min_angle: float = 25.0,
) -> Mesh:
    """Photonic-crystal-fibre cross-section: disk of radius ``R`` whose mesh conforms
    to a hexagonal lattice of circular holes (central hole removed)."""
    centres = pcf_hole_centres(pitch, n_rings)

    def build(rng):
        p = _hex_lattice(-R, R, -R, R, h)
        p = p + rng.uniform(-jitter * h, jitter * h, p.shape)
        keep = np.hypot(p[:, 0], p[:, 1]) <= R - 0.75 * h
        for cx, cy in centres:
            d = np.hypot(p[:, 0] - cx, p[:, 1] - cy)
            keep &= np.abs(d - hole_radius) >= 0.75 * h
        parts = [p[keep], _ring(R, round(2 * math.pi * R / h), rng)]
        for cx, cy in centres:
            parts.append(_ring(hole_radius, round(2 * math.pi * hole_radius / h), rng, centre=(cx, cy)))
        meta = {"kind": "pcf", "R": R, "h": h, "hole_radius": hole_radius, "pitch": pitch, "n_rings": n_rings,
                "hole_centres": centres}
        return _finish(np.concatenate(parts), meta, min_angle)

    return _retry(build, seed, min_angle)


def regular_grid_mesh(nx: int, ny: int, hx: float, hy: float | None = None, x0: float = 0.0, y0: float = 0.0,
                      flip: bool = False) -> Mesh:
    """Structured grid of ``nx`` by ``ny`` vertices, each cell split into two right
    triangles along the same diagonal (listed counter-clockwise)."""
    hy = hx if hy is None else hy
    X, Y = np.meshgrid(x0 + hx * np.arange(nx), y0 + hy * np.arange(ny), indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    idx = np.arange(nx * ny).reshape(ny, nx)
    a = idx[:-1, :-1].ravel()
    b = idx[:-1, 1:].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[1:, :-1].ravel()
    if not flip:
        tri = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    else:
        tri = np.concatenate([np.stack([a, b, d], 1), np.stack([b, c, d], 1)])
    return Mesh(xy, tri.astype(np.int32), {"kind": "grid", "hx": hx, "hy": hy, "nx": nx, "ny": ny})


def strip_mesh(L: float, h: float, n_rows: int = 4) -> Mesh:
    """Right-triangle strip ``[-L, L] x [0, (n_rows-1) h]`` for quasi-1D tests."""
    nx = int(round(2 * L / h)) + 1
    return regular_grid_mesh(nx, n_rows, h, h, x0=-L, y0=0.0)


def hex_patch_mesh(h: float = 1.0, rings: int = 1) -> Mesh:
    """Equilateral hexagonal patch (a centre vertex and ``rings`` hexagonal rings)."""
    pts = [(0.0, 0.0)]
    for k in range(1, rings + 1):
        for s in range(6):
            a0 = math.pi / 3 * s
            a1 = math.pi / 3 * (s + 1)
            p0 = np.array([math.cos(a0), math.sin(a0)]) * k * h
            p1 = np.array([math.cos(a1), math.sin(a1)]) * k * h
            for j in range(k):
                pts.append(tuple(p0 + (p1 - p0) * j / k))
    pts = np.array(pts)
    return Mesh(pts, _triangulate(pts), {"kind": "hex_patch", "h": h, "rings": rings})


def random_delaunay_mesh(n: int, seed: int, min_angle: float = 0.0) -> Mesh:
    """Delaunay triangulation of ``n`` uniform random points in the unit square
    (any quality; for structure tests)."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, (n, 2))
    mesh, _ = _finish(pts, {"kind": "random", "n": n}, min_angle)
    return mesh


def wheel_disk_mesh(R: float = 10.0, h: float = 0.3, seed: int = 5, spokes: int = 14,
                    centres=((0.0, 0.0), (3.0, 2.0)), min_angle: float = 25.0) -> Mesh:
    """Disk of radius ``R`` (as ``disk_mesh``) with a wheel around each centre: the
    centre vertex, ``spokes`` points on a circle of radius ``h`` and a second
    ring at ``1.8 h`` (half a spoke out of phase), the lattice cleared within
    ``2.4 h``.  The centres get degree ``spokes``: 14 is the most a vertex can
    have while every angle stays at least 25 degrees (360/14 = 25.7)."""
    spacing = 2.0 * math.pi * h / spokes

    def build(rng):
        p = _hex_lattice(-R, R, -R, R, h)
        p = p + rng.uniform(-0.05 * h, 0.05 * h, p.shape)
        p = p[np.hypot(p[:, 0], p[:, 1]) < R - 0.75 * h]
        for c in centres:
            p = p[np.hypot(p[:, 0] - c[0], p[:, 1] - c[1]) > 2.4 * h]
        parts = [p, _ring(R, round(2.0 * math.pi * R / h), rng)]
        for c in centres:
            parts.append(np.array([c], dtype=np.float64))
            parts.append(_ring(h, spokes, rng, centre=c, phase=0.0))
            parts.append(_ring(1.8 * h, round(0.55 * 2.0 * math.pi * 1.8 * h / spacing), rng, centre=c,
                               phase=math.pi / spokes))
        return _finish(np.concatenate(parts), {"kind": "wheel_disk", "R": R, "h": h, "spokes": spokes}, min_angle)

    return _retry(build, seed, min_angle)


def jittered_lattice_mesh(nx: int, ny: int, jitter: float, seed: int, angle: float = 0.0, shear: float = 0.0,
                          shuffle: bool = True) -> Mesh:
    """Delaunay triangulation of an ``nx`` x ``ny`` hexagonal lattice (spacing 1),
    each point moved by up to ``jitter`` in each coordinate, then sheared by
    ``shear`` and rotated by ``angle``; with ``shuffle`` the vertex order, the
    triangle order and each triangle's orientation are randomised (seeded), as
    an arbitrary mesher's output would be.  For property tests of mesh ingest.
    Without jitter the lattice's straight rows give Qhull collinear (zero-area)
    triangles on the hull, which a valid mesh cannot have: use jitter > 0."""
    rng = np.random.default_rng(seed)
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = ii + 0.5 * (jj & 1)
    y = jj * (math.sqrt(3.0) / 2.0)
    pts = np.stack([x.ravel(), y.ravel()], axis=1).astype(np.float64)
    pts = pts + rng.uniform(-jitter, jitter, pts.shape)
    pts[:, 0] += shear * pts[:, 1]
    c, s_ = math.cos(angle), math.sin(angle)
    pts = pts @ np.array([[c, s_], [-s_, c]])
    tri = _triangulate(pts)
    if shuffle:
        order = rng.permutation(len(pts))
        inv = np.empty_like(order)
        inv[order] = np.arange(len(pts))
        pts = pts[order]
        tri = inv[tri].astype(np.int32)
        tri = tri[rng.permutation(len(tri))]
        flip = rng.random(len(tri)) < 0.5
        tri[flip] = tri[flip][:, [0, 2, 1]]
    meta = {"kind": "jittered_lattice", "nx": nx, "ny": ny, "jitter": jitter, "seed": seed,
            "min_angle_deg": min_angle_deg(pts, tri)}
    return Mesh(np.ascontiguousarray(pts), np.ascontiguousarray(tri, dtype=np.int32), meta)
