"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module builds only *inputs* of the solver: tetrahedral meshes (vertex ids and
coordinates), per-tet velocity / quality factor samples, boundary tags, subdomain
partitions, coarse meshes and source positions.  It holds none of the method's
arithmetic (no basis functions, no element integrals, no assembly, no solver).

Mesh family.  A structured box of nx*ny*nz cubes, each cut into six tetrahedra along
its main diagonal (Kuhn / Freudenthal split).  The paper runs on unstructured meshes
of the SEG/EAGE Overthrust box (section "Numerical results"); that model is not
available, so a layered synthetic velocity model on the same 20 x 20 x 4.65 km box
stands in for it (velocity 2.2-6.0 km/s, free surface on top, absorbing elsewhere).

Conventions
* vertex id      = i + (nx+1)*(j + (ny+1)*k)
* cube id        = i + nx*(j + ny*k)
* tet id         = 6*cube + p, with p indexing the axis permutation
                   (0,1,2),(0,2,1),(1,0,2),(1,2,0),(2,0,1),(2,1,0); the tet's vertices are
                   c, c+e[p0], c+e[p0]+e[p1], c+(1,1,1)
* z points down, z = 0 is the free surface.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BC_NONE, BC_IMPEDANCE, BC_DIRICHLET = 0, 1, 2

_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn_mesh(xs, ys, zs):
    """Six-tet Kuhn mesh of the tensor grid xs x ys x zs (1-D coordinate arrays)."""
    xs = np.asarray(xs, np.float64)
    ys = np.asarray(ys, np.float64)
    zs = np.asarray(zs, np.float64)
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    coords = np.stack([xs[ii.ravel()], ys[jj.ravel()], zs[kk.ravel()]], axis=1)

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    ncube = ci.size
    tets = np.empty((ncube, 6, 4), np.int64)
    for p, perm in enumerate(_PERMS):
        off = np.zeros(3, np.int64)
        verts = [vid(ci, cj, ck)]
        for ax in perm[:2]:
            off[ax] += 1
            verts.append(vid(ci + off[0], cj + off[1], ck + off[2]))
        verts.append(vid(ci + 1, cj + 1, ck + 1))
        tets[:, p, :] = np.stack(verts, axis=1)
    return tets.reshape(-1, 4).astype(np.int32), coords


def tet_centroids(tets, coords):
    return coords[tets].mean(axis=1)


def face_bc_tags(tets, coords, dirichlet_top=True, ztop=0.0):
    """Per (tet, local face) boundary tag; local face f is the face opposite local vertex f.

    Tags are read by the solver only on boundary faces (faces of a single tet).  Faces
    lying in the plane z = ztop are Dirichlet (free surface) when dirichlet_top, every
    other face is impedance (first-order absorbing)."""
    tags = np.full((tets.shape[0], 4), BC_IMPEDANCE, np.int8)
    if dirichlet_top:
        onz = np.abs(coords[:, 2] - ztop) <= 1e-9 * max(1.0, float(np.abs(coords[:, 2]).max()))
        vz = onz[tets]  # (T, 4)
        for f in range(4):
            others = [v for v in range(4) if v != f]
            tags[vz[:, others].all(axis=1), f] = BC_DIRICHLET
    return tags


def box_partition(nx, ny, nz, px, py, pz, xcuts=None, ycuts=None, zcuts=None):
    """Subdomain id per tet from the index of its cube in a px*py*pz grid of boxes.

    Default cuts split each axis into near-equal cube counts; explicit cut arrays
    (cube indices, length p+1) allow uneven boxes.  id = bx + px*(by + py*bz)."""

    def cuts(n, p, c):
        if c is None:
            c = np.round(np.linspace(0, n, p + 1)).astype(np.int64)
        return np.asarray(c, np.int64)

    cx, cy, cz = cuts(nx, px, xcuts), cuts(ny, py, ycuts), cuts(nz, pz, zcuts)
    bx = np.searchsorted(cx, np.arange(nx), side="right") - 1
    by = np.searchsorted(cy, np.arange(ny), side="right") - 1
    bz = np.searchsorted(cz, np.arange(nz), side="right") - 1
    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    part_cube = bx[ci.ravel()] + px * (by[cj.ravel()] + py * bz[ck.ravel()])
    return np.repeat(part_cube, 6).astype(np.int32)


# --------------------------------------------------------------------------- model


@dataclass
class LayeredModel:
    """v0(z) = 2200 + 3800 z/4.65 (m/s, z in km) with 12 Gaussian anomalies of +-10 %
    and 3 dipping step layers, all drawn from numpy PCG64(seed)."""

    seed: int = 2004
    lx: float = 20.0
    ly: float = 20.0
    lz: float = 4.65
    anomalies: list = field(default_factory=list)
    layers: list = field(default_factory=list)

    def __post_init__(self):
        rng = np.random.Generator(np.random.PCG64(self.seed))
        self.anomalies = []
        for _ in range(12):
            c = rng.uniform([0, 0, 0], [self.lx, self.ly, self.lz])
            r = rng.uniform(0.5, 2.0)
            sgn = 1.0 if rng.uniform() < 0.5 else -1.0
            self.anomalies.append((c, r, sgn))
        self.layers = []
        for _ in range(3):
            zl = rng.uniform(1.0, 4.0)
            th = math.radians(rng.uniform(5.0, 20.0))
            ph = rng.uniform(0.0, 2 * math.pi)
            dv = rng.uniform(150.0, 400.0)
            self.layers.append((zl, th, ph, dv))

    def v0(self, z_km):
        return 2200.0 + 3800.0 * np.asarray(z_km) / self.lz

    def velocity(self, x_km, y_km, z_km):
        x, y, z = (np.asarray(a, np.float64) for a in (x_km, y_km, z_km))
        v = self.v0(z).astype(np.float64)
        for zl, th, ph, dv in self.layers:
            plane = zl + math.tan(th) * ((x - self.lx / 2) * math.cos(ph) + (y - self.ly / 2) * math.sin(ph))
            v = v + np.where(z > plane, dv, 0.0)
        for c, r, sgn in self.anomalies:
            d2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
            v = v * (1.0 + sgn * 0.10 * np.exp(-d2 / (r * r)))
        return v

    def quality(self, z_km):
        return 80.0 + 120.0 * np.asarray(z_km) / self.lz


def graded_layers(model: LayeredModel, freq, r, multiple=4):
    """Depth nodes (km) for layers of thickness h_z(z) = 0.9 v0(z) / (2 f r).

    The layer count N = ceil(int_0^lz dz / h_z) is rounded up to a multiple of
    `multiple`, and the nodes are placed at equal steps of travel time
    tau(z) = int_0^z dz / v0 so that h_z stays proportional to v0 and the last node is
    exactly the bottom of the box."""
    a, b = 2200.0, 3800.0 / model.lz  # v0 = a + b z  (m/s, z in km)
    tau = lambda z: math.log((a + b * z) / a) / b  # km*s/m
    ttot = tau(model.lz)
    n = int(math.ceil(2.0 * freq * r / 0.9 * ttot * 1000.0 - 1e-9))
    n = int(math.ceil(n / multiple) * multiple)
    t = ttot * np.arange(n + 1) / n
    zs = (a / b) * (np.exp(b * t) - 1.0)
    zs[0], zs[-1] = 0.0, model.lz
    return zs


@dataclass
class Problem:
    """Everything the solver takes as input for one operator."""

    name: str
    tets: np.ndarray
    coords: np.ndarray
    face_bc: np.ndarray
    velocity: np.ndarray
    quality: np.ndarray | None
    freq: float
    partition: np.ndarray
    n_sub: int
    overlap: int
    coarse_tets: np.ndarray | None = None
    coarse_coords: np.ndarray | None = None
    sources: np.ndarray | None = None  # (ns, 3) in the mesh's length unit
    grid: tuple = ()
    tol: float = 1e-6
    extra: dict = field(default_factory=dict)


def plane_wave_direction(seed=1):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal(3)
    return g / np.linalg.norm(g)


def unit_cube_problem(n=8, freq=4.0, parts=(2, 2, 2), overlap=1, seed=1):
    """Unit cube, n^3 cubes x 6 tets, v = 1, impedance on every face, box partition."""
    xs = np.linspace(0.0, 1.0, n + 1)
    tets, coords = kuhn_mesh(xs, xs, xs)
    T = tets.shape[0]
    px, py, pz = parts
    part = box_partition(n, n, n, px, py, pz)
    return Problem(
        name=f"unit_cube_{n}",
        tets=tets,
        coords=coords,
        face_bc=face_bc_tags(tets, coords, dirichlet_top=False),
        velocity=np.ones(T),
        quality=None,
        freq=freq,
        partition=part,
        n_sub=px * py * pz,
        overlap=overlap,
        grid=(n, n, n),
        tol=1e-8,
        extra={"direction": plane_wave_direction(seed)},
    )


def layered_problem(freq=2.5, r=1.4, parts=(8, 8, 1), overlap=2, n_sources=(4, 4), src_depth=0.5,
                    lateral=None, with_q=False, coarse_factor=4, seed=2004, xy_multiple=4,
                    equal_depth_zcuts=False, max_cubes=None):
    """Layered synthetic model on the 20 x 20 x 4.65 km box (lengths in km).

    Horizontal cube size lambda_min/(2r) with lambda_min = 1980/f m; vertical layers graded
    with the background velocity; counts rounded up to multiples of xy_multiple (the
    coarse grid takes every coarse_factor-th vertex plane).  `lateral` = (x0, x1, y0, y1)
    restricts the box to a lateral window (one GPU's block of a larger domain).
    `max_cubes` caps (nx, ny) for scaled-down variants of the same family."""
    model = LayeredModel(seed=seed)
    lam_min = 1980.0 / freq / 1000.0  # km
    hxy = lam_min / (2.0 * r)
    x0, x1, y0, y1 = lateral if lateral is not None else (0.0, model.lx, 0.0, model.ly)
    nx = int(math.ceil((x1 - x0) / hxy / xy_multiple) * xy_multiple)
    ny = int(math.ceil((y1 - y0) / hxy / xy_multiple) * xy_multiple)
    if max_cubes is not None:
        nx, ny = min(nx, max_cubes[0]), min(ny, max_cubes[1])
    zs = graded_layers(model, freq, r, multiple=xy_multiple)
    if max_cubes is not None and len(max_cubes) > 2:
        nzc = max_cubes[2]
        zs = np.interp(np.linspace(0, len(zs) - 1, nzc + 1), np.arange(len(zs)), zs)
    nz = len(zs) - 1
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    tets, coords = kuhn_mesh(xs, ys, zs)
    cen = tet_centroids(tets, coords)
    vel = model.velocity(cen[:, 0], cen[:, 1], cen[:, 2])
    q = model.quality(cen[:, 2]) if with_q else None
    px, py, pz = parts
    zc = None
    if equal_depth_zcuts and pz > 1:
        zc = np.searchsorted(zs, np.linspace(0, model.lz, pz + 1)[1:-1])
        zc = np.concatenate([[0], zc, [nz]])
    part = box_partition(nx, ny, nz, px, py, pz, zcuts=zc)
    ctets = ccoords = None
    if coarse_factor and nx % coarse_factor == 0 and ny % coarse_factor == 0 and nz % coarse_factor == 0:
        ctets, ccoords = kuhn_mesh(xs[::coarse_factor], ys[::coarse_factor], zs[::coarse_factor])
    sx, sy = n_sources
    srcx = x0 + (np.arange(sx) + 0.5) * (x1 - x0) / sx
    srcy = y0 + (np.arange(sy) + 0.5) * (y1 - y0) / sy
    gx, gy = np.meshgrid(srcx, srcy, indexing="ij")
    src = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, src_depth)], axis=1)
    return Problem(
        name=f"layered_{freq}Hz",
        tets=tets,
        coords=coords,
        face_bc=face_bc_tags(tets, coords, dirichlet_top=True),
        velocity=vel * 1e-3,  # km/s, consistent with lengths in km
        quality=q,
        freq=freq,
        partition=part,
        n_sub=px * py * pz,
        overlap=overlap,
        coarse_tets=ctets,
        coarse_coords=ccoords,
        sources=src,
        grid=(nx, ny, nz),
        tol=1e-6,
        extra={"r": r, "parts": tuple(parts)},
    )


def kuhn_ndofs(nx, ny, nz):
    return (3 * nx + 1) * (3 * ny + 1) * (3 * nz + 1)


def seeded_rhs_block(n, s, seed):
    """Dense complex right-hand sides with standard normal parts, shape (s, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((s, n)) + 1j * rng.standard_normal((s, n))
