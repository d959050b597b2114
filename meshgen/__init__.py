"""Seeded synthetic surface meshes (inputs only).

This module builds the closed, oriented triangle meshes that both the CPU
oracle and the GPU library consume.  It holds none of the loop-shrinking
method's arithmetic: no field, threshold, front or event logic lives here,
only geometry generation (parametric torus, signed-distance surfaces
extracted by marching tetrahedra), vertex welding, jitter and seed choice.

Every mesh is returned as ``Mesh(xyz float64[V,3], tri int32[F,3], seed)``
with triangles oriented so that their normals point out of the solid
(counter-clockwise seen from outside).

Workloads (the paper's detailed scanned models are not available, so these
synthetic surfaces of known genus stand in for them):

* ``torus_grid``      -- 64x32 parametric torus, R=1, r=0.4, N(0,1e-3) jitter
* ``pretzel``         -- genus-3 union of three tori (R=1, r=0.35, centres
                         x=-1.6,0,1.6), level-0 surface on a 256^3 sample grid
                         fitted per axis to the bounding box plus 2 cells,
                         N(0,1e-4) jitter
* ``sdf_surface``     -- any signed-distance function at any grid size
                         (small spheres, tori, multi-tori for tests)
* ``uv_sphere``       -- latitude-longitude sphere whose poles have high
                         degree (tests of wide vertices)
* ``voxel_surface``   -- unjittered boundary of a set of unit voxels; the
                         exact symmetry of such surfaces makes fronts meet
                         in ties (3-way merges, 1-to-3 splits, monkey
                         saddles)
* ``csaszar_torus``   -- the 7-vertex torus (every vertex adjacent to every
                         other one)
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Mesh", "torus_grid", "marching_tets", "sdf_surface", "pretzel", "batch_workload",
    "sdf_sphere", "sdf_torus", "sdf_union_tori", "sdf_box", "jittered",
    "pick_seed", "euler_characteristic", "pretzel_sdf", "multi_torus", "uv_sphere",
    "voxel_surface", "voxel_frame", "csaszar_torus", "octahedron", "icosphere", "relaxed",
]


@dataclass
class Mesh:
    xyz: np.ndarray          # float64 [V,3]
    tri: np.ndarray          # int32   [F,3], outward oriented
    seed: int = 0            # seed vertex chosen from the generator's PRNG
    name: str = ""

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nf(self) -> int:
        return int(self.tri.shape[0])


def euler_characteristic(tri: np.ndarray, nv: int) -> int:
    """V - E + F of a triangle mesh (edges counted once)."""
    t = np.asarray(tri, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e.sort(axis=1)
    ne = np.unique(e[:, 0] * nv + e[:, 1]).size
    return int(nv - ne + t.shape[0])


# ---------------------------------------------------------------------------
# parametric torus
# ---------------------------------------------------------------------------
def torus_grid(n_major: int = 64, n_minor: int = 32, R: float = 1.0,
               r: float = 0.4, jitter: float = 1e-3, rng_seed: int = 0,
               jitter_first: bool = True) -> Mesh:
    """Regular torus grid: vertex (i,j) has id ``n_minor*i + j`` and sits at
    ((R + r cos phi_j) cos th_i, (R + r cos phi_j) sin th_i, r sin phi_j),
    th_i = 2 pi i / n_major, phi_j = 2 pi j / n_minor.  Each grid quad
    (i,j),(i+1,j),(i+1,j+1),(i,j+1) is split along its (i,j)-(i+1,j+1)
    diagonal.  One PRNG stream draws the N(0, jitter^2) coordinate noise
    first, then the seed vertex."""
    i = np.arange(n_major)
    j = np.arange(n_minor)
    th = 2.0 * np.pi * i / n_major
    ph = 2.0 * np.pi * j / n_minor
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    x = (R + r * np.cos(PH)) * np.cos(TH)
    y = (R + r * np.cos(PH)) * np.sin(TH)
    z = r * np.sin(PH)
    xyz = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)
    I, J = np.meshgrid(i, j, indexing="ij")
    I = I.ravel()
    J = J.ravel()
    I1 = (I + 1) % n_major
    J1 = (J + 1) % n_minor
    v00 = n_minor * I + J
    v10 = n_minor * I1 + J
    v11 = n_minor * I1 + J1
    v01 = n_minor * I + J1
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    tri = np.empty((2 * t1.shape[0], 3), dtype=np.int32)
    tri[0::2] = t1
    tri[1::2] = t2
    rng = np.random.default_rng(rng_seed)
    xyz = xyz + rng.normal(0.0, jitter, size=xyz.shape)
    seed = int(rng.integers(xyz.shape[0]))
    return Mesh(xyz, tri, seed, f"torus{n_major}x{n_minor}")


def uv_sphere(n_lat: int = 30, n_lon: int = 40, jitter: float = 1e-3, rng_seed: int = 0) -> Mesh:
    """Latitude-longitude unit sphere: the north pole (id 0), n_lat rings of
    n_lon vertices (ring r, column c -> id 1 + n_lon*r + c, colatitude
    pi (r+1)/(n_lat+1), longitude 2 pi c/n_lon), the south pole (last id).
    The poles have degree n_lon, the vertices of the two rings next to them
    5, all others 6; genus 0.  One PRNG stream draws the N(0, jitter^2)
    coordinate noise, then the seed."""
    r = np.arange(n_lat)
    c = np.arange(n_lon)
    th = np.pi * (r + 1) / (n_lat + 1)
    ph = 2.0 * np.pi * c / n_lon
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    ring = np.stack([(np.sin(TH) * np.cos(PH)).ravel(), (np.sin(TH) * np.sin(PH)).ravel(),
                     np.cos(TH).ravel()], axis=1)
    xyz = np.concatenate([[[0.0, 0.0, 1.0]], ring, [[0.0, 0.0, -1.0]]]).astype(np.float64)
    S = 1 + n_lat * n_lon

    def vid(rr, cc):
        return 1 + n_lon * rr + (cc % n_lon)

    tris = []
    for cc in range(n_lon):
        tris.append((0, vid(0, cc), vid(0, cc + 1)))
        tris.append((S, vid(n_lat - 1, cc + 1), vid(n_lat - 1, cc)))
    for rr in range(n_lat - 1):
        for cc in range(n_lon):
            a, b, e, d = vid(rr, cc), vid(rr + 1, cc), vid(rr + 1, cc + 1), vid(rr, cc + 1)
            tris.append((a, b, e))
            tris.append((a, e, d))
    tri = np.array(tris, dtype=np.int32)
    rng = np.random.default_rng(rng_seed)
    xyz = xyz + rng.normal(0.0, jitter, size=xyz.shape)
    seed = int(rng.integers(xyz.shape[0]))
    return Mesh(xyz, tri, seed, f"uvsphere{n_lat}x{n_lon}")


def octahedron(radius: float = 1.0, rng_seed: int = 0) -> Mesh:
    """Regular octahedron (8 equilateral faces, every vertex of valence 4),
    outward oriented; the seed vertex from the PRNG."""
    xyz = radius * np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                            dtype=np.float64)
    tri = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                    [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int32)
    seed = int(np.random.default_rng(rng_seed).integers(6))
    return Mesh(xyz, tri, seed, "octahedron")


def icosphere(subdiv: int = 0, radius: float = 1.0, rng_seed: int = 0) -> Mesh:
    """Regular icosahedron (subdiv 0: 20 equilateral faces, every vertex of
    valence 5), each further level splitting every triangle into four and
    projecting the new vertices onto the sphere; outward oriented; the seed
    vertex from the PRNG."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    xyz = [[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
           [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]]
    xyz = [list(np.asarray(p, dtype=np.float64) / np.linalg.norm(p)) for p in xyz]
    tri = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4], [11, 10, 2],
           [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5],
           [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    for _ in range(subdiv):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                p = np.asarray(xyz[a]) + np.asarray(xyz[b])
                xyz.append(list(p / np.linalg.norm(p)))
                mid[key] = len(xyz) - 1
            return mid[key]
        nt = []
        for a, b, c in tri:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nt += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        tri = nt
    xyz = radius * np.asarray(xyz, dtype=np.float64)
    seed = int(np.random.default_rng(rng_seed).integers(xyz.shape[0]))
    return Mesh(xyz, np.asarray(tri, dtype=np.int32), seed, f"icosphere{subdiv}")


def relaxed(m: Mesh, f, iters: int = 10, lam: float = 0.5, h: float = 1e-6) -> Mesh:
    """Better-shaped triangles on the same surface, for the finite-element
    operator (marching-tetrahedra slivers make its coefficients, and so its
    stable explicit step, extreme): ``iters`` rounds of moving every vertex
    a fraction ``lam`` towards the mean of its neighbours, then three Newton
    steps back onto the level 0 of the distance function ``f`` (central
    differences of step ``h``).  Connectivity, and so the genus, is kept."""
    import scipy.sparse as sp
    xyz = m.xyz.copy()
    nv = xyz.shape[0]
    t = m.tri.astype(np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    A = sp.coo_matrix((np.ones(e.shape[0]), (e[:, 0], e[:, 1])), shape=(nv, nv)).tocsr()
    A = ((A + A.T) > 0).astype(np.float64)
    deg = np.asarray(A.sum(axis=1)).ravel()
    for _ in range(iters):
        xyz = xyz + lam * ((A @ xyz) / deg[:, None] - xyz)
        for _ in range(3):
            x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
            fx = f(x, y, z)
            g = np.stack([(f(x + h, y, z) - f(x - h, y, z)) / (2 * h),
                          (f(x, y + h, z) - f(x, y - h, z)) / (2 * h),
                          (f(x, y, z + h) - f(x, y, z - h)) / (2 * h)], axis=1)
            xyz = xyz - (fx / np.maximum((g * g).sum(axis=1), 1e-30))[:, None] * g
    return Mesh(xyz, m.tri, m.seed, (m.name or "mesh") + f"_relaxed{iters}")


# ---------------------------------------------------------------------------
# signed distance functions (negative inside the solid)
# ---------------------------------------------------------------------------
def sdf_sphere(c=(0.0, 0.0, 0.0), rad=1.0):
    c = np.asarray(c, dtype=np.float64)

    def f(x, y, z):
        return np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) - rad
    return f


def sdf_torus(c=(0.0, 0.0, 0.0), R=1.0, r=0.35):
    """Torus in the xy-plane around centre c."""
    c = np.asarray(c, dtype=np.float64)

    def f(x, y, z):
        q = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2) - R
        return np.sqrt(q * q + (z - c[2]) ** 2) - r
    return f


def sdf_union_tori(centres, R=1.0, r=0.35):
    parts = [sdf_torus(c, R, r) for c in centres]

    def f(x, y, z):
        out = parts[0](x, y, z)
        for p in parts[1:]:
            out = np.minimum(out, p(x, y, z))
        return out
    return f


def sdf_box(half=(1.0, 1.0, 1.0)):
    h = np.asarray(half, dtype=np.float64)

    def f(x, y, z):
        qx = np.abs(x) - h[0]
        qy = np.abs(y) - h[1]
        qz = np.abs(z) - h[2]
        outside = np.sqrt(np.maximum(qx, 0) ** 2 + np.maximum(qy, 0) ** 2 +
                          np.maximum(qz, 0) ** 2)
        inside = np.minimum(np.maximum(qx, np.maximum(qy, qz)), 0.0)
        return outside + inside
    return f


# ---------------------------------------------------------------------------
# marching tetrahedra
# ---------------------------------------------------------------------------
# Corner (dx,dy,dz) of a grid cell has local index dx + 2 dy + 4 dz.  The cell
# is cut into 6 tetrahedra along its main diagonal 000-111 (one per ordering
# of the three axes); neighbouring cells then agree on every shared face
# diagonal, so the extracted surface is watertight.
def _cell_tets():
    tets = []
    for perm in itertools.permutations(range(3)):
        p = [0, 0, 0]
        corners = [0]
        for ax in perm:
            p[ax] = 1
            corners.append(p[0] + 2 * p[1] + 4 * p[2])
        # orientation sign of (e_p0, e_p0+e_p1, e_p0+e_p1+e_p2) = parity(perm)
        inv = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b])
        if inv % 2 == 1:
            corners[2], corners[3] = corners[3], corners[2]
        tets.append(corners)
    return np.array(tets, dtype=np.int64)          # [6,4], positive volume


def _even(p):
    inv = sum(1 for a in range(4) for b in range(a + 1, 4) if p[a] > p[b])
    return inv % 2 == 0


def _tet_case_table():
    """For each of the 16 inside-patterns of a positively oriented tet
    (bit i set = local vertex i inside), up to two triangles, each given by
    three tet edges (pairs of local vertex indices), oriented so the normal
    points from the inside vertices toward the outside ones."""
    table = np.full((16, 2, 3, 2), -1, dtype=np.int64)
    ntri = np.zeros(16, dtype=np.int64)
    for case in range(16):
        ins = [i for i in range(4) if case >> i & 1]
        outs = [i for i in range(4) if not case >> i & 1]
        if len(ins) in (0, 4):
            continue
        if len(ins) in (1, 3):
            lone = ins[0] if len(ins) == 1 else outs[0]
            rest = [i for i in range(4) if i != lone]
            p = [lone] + rest
            if not _even(p):
                p = [lone, rest[1], rest[0], rest[2]]
            a, b, c, d = p
            tri = [(a, b), (a, c), (a, d)]          # normal points away from a
            if len(ins) == 3:                       # a is outside: flip
                tri = [tri[0], tri[2], tri[1]]
            table[case, 0] = tri
            ntri[case] = 1
        else:
            p = ins + outs
            if not _even(p):
                p = [ins[0], ins[1], outs[1], outs[0]]
            a, b, c, d = p
            table[case, 0] = [(a, c), (a, d), (b, d)]
            table[case, 1] = [(a, c), (b, d), (b, c)]
            ntri[case] = 2
    return table, ntri


_TETS = _cell_tets()
_CASES, _NTRI = _tet_case_table()


def marching_tets(f, lo, hi, shape, chunk_cells: int = 1 << 21) -> Mesh:
    """Level-0 surface of ``f`` sampled on a regular grid of ``shape`` points
    spanning [lo, hi] (per axis).  Inside means f < 0; a sample equal to 0
    counts as outside.  Vertices sit on crossed tet edges at the linear
    interpolation of f and are welded by their grid-edge key, then numbered
    in ascending key order (grid order, spatially local)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    nx, ny, nz = (int(s) for s in shape)
    h = (hi - lo) / (np.array([nx, ny, nz], dtype=np.float64) - 1.0)
    xs = lo[0] + h[0] * np.arange(nx)
    ys = lo[1] + h[1] * np.arange(ny)
    zs = lo[2] + h[2] * np.arange(nz)
    # grid point (i,j,k) -> linear id i*ny*nz + j*nz + k
    F = np.empty((nx, ny, nz), dtype=np.float64)
    Y, Z = np.meshgrid(ys, zs, indexing="ij")
    for i in range(nx):
        F[i] = f(np.full_like(Y, xs[i]), Y, Z)
    neg = F < 0
    # cells with a sign change among their 8 corners
    c = neg[:-1, :-1, :-1].astype(np.int8)
    anyin = np.zeros((nx - 1, ny - 1, nz - 1), dtype=bool)
    allin = np.ones((nx - 1, ny - 1, nz - 1), dtype=bool)
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                s = neg[dx:nx - 1 + dx, dy:ny - 1 + dy, dz:nz - 1 + dz]
                anyin |= s
                allin &= s
    del c
    cells = np.flatnonzero(anyin & ~allin)
    del anyin, allin
    ci, rem = np.divmod(cells, (ny - 1) * (nz - 1))
    cj, ck = np.divmod(rem, nz - 1)
    base = ci * ny * nz + cj * nz + ck
    corner_off = np.array([dx * ny * nz + dy * nz + dz
                           for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)],
                          dtype=np.int64)
    # corner_off index = dx + 2dy + 4dz
    Ff = F.ravel()
    negf = neg.ravel()
    keys_all = []
    for s0 in range(0, base.size, chunk_cells):
        b = base[s0:s0 + chunk_cells]
        for t in range(6):
            g = b[:, None] + corner_off[_TETS[t]][None, :]      # [n,4] grid ids
            ins = negf[g]
            case = ins[:, 0] * 1 + ins[:, 1] * 2 + ins[:, 2] * 4 + ins[:, 3] * 8
            for k in (0, 1):
                sel = _NTRI[case] > k
                if not np.any(sel):
                    continue
                cs = case[sel]
                gs = g[sel]
                e = _CASES[cs, k]                                # [m,3,2]
                ga = np.take_along_axis(gs, e[:, :, 0], axis=1)
                gb = np.take_along_axis(gs, e[:, :, 1], axis=1)
                kmin = np.minimum(ga, gb)
                kmax = np.maximum(ga, gb)
                keys_all.append(kmin * (nx * ny * nz) + kmax)    # [m,3]
    keys = np.concatenate(keys_all, axis=0)
    uk, inv = np.unique(keys.ravel(), return_inverse=True)
    tri = inv.reshape(-1, 3).astype(np.int32)
    npts = nx * ny * nz
    ga = uk // npts
    gb = uk % npts
    fa = Ff[ga]
    fb = Ff[gb]
    t = fa / (fa - fb)

    def coords(gid):
        i, r = np.divmod(gid, ny * nz)
        j, k = np.divmod(r, nz)
        return np.stack([xs[i], ys[j], zs[k]], axis=1)
    pa = coords(ga)
    pb = coords(gb)
    xyz = pa + t[:, None] * (pb - pa)
    return Mesh(xyz.astype(np.float64), tri, 0, "mt")


def jittered(m: Mesh, sigma: float, rng_seed: int, name: str = "") -> Mesh:
    """N(0, sigma^2) coordinate noise, then a seed vertex, from one stream."""
    rng = np.random.default_rng(rng_seed)
    xyz = m.xyz + rng.normal(0.0, sigma, size=m.xyz.shape)
    seed = int(rng.integers(m.nv))
    return Mesh(xyz, m.tri, seed, name or m.name)


def pick_seed(m: Mesh, rng_seed: int) -> Mesh:
    rng = np.random.default_rng(rng_seed)
    return Mesh(m.xyz, m.tri, int(rng.integers(m.nv)), m.name)


def _fitted_grid(lo, hi, n, margin=2):
    """Per-axis sample grid of n points covering [lo,hi] with ``margin``
    empty cells on each side."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    n = np.asarray(n, dtype=np.int64)
    h = (hi - lo) / (n - 1 - 2 * margin)
    return lo - margin * h, hi + margin * h


def sdf_surface(f, lo, hi, n, sigma=0.0, rng_seed=0, name="", margin=2):
    if np.isscalar(n):
        n = (n, n, n)
    glo, ghi = _fitted_grid(lo, hi, n, margin)
    m = marching_tets(f, glo, ghi, n)
    return jittered(m, sigma, rng_seed, name)


PRETZEL_CENTRES = ((-1.6, 0.0, 0.0), (0.0, 0.0, 0.0), (1.6, 0.0, 0.0))


def pretzel_sdf(R=1.0, r=0.35):
    return sdf_union_tori(PRETZEL_CENTRES, R, r)


def multi_torus(g: int, n: int, R: float = 1.0, r: float = 0.35,
                spacing: float = 1.6, sigma: float = 1e-4, rng_seed: int = 0) -> Mesh:
    """Chain of ``g`` tori at ``spacing`` along x (genus g for g>=1 with
    spacing < 2R), level-0 surface on an n^3 grid fitted per axis."""
    cx = (np.arange(g) - (g - 1) / 2.0) * spacing
    centres = [(float(x), 0.0, 0.0) for x in cx]
    f = sdf_union_tori(centres, R, r)
    lo = (cx[0] - R - r, -R - r, -r)
    hi = (cx[-1] + R + r, R + r, r)
    return sdf_surface(f, lo, hi, n, sigma, rng_seed, f"torus_chain{g}_{n}")


def pretzel(n: int = 256, sigma: float = 1e-4, rng_seed: int = 0) -> Mesh:
    """Genus-3 pretzel: level 0 of min over three tori SDFs (R=1, r=0.35,
    centres x = -1.6, 0, 1.6), n samples per axis fitted to the bounding box
    plus two cells, N(0, sigma^2) jitter, then a seed vertex."""
    return multi_torus(3, n, 1.0, 0.35, 1.6, sigma, rng_seed)


def batch_workload(n: int = 1024, base_seed: int = 0, pretzel_grids=(32, 48, 64, 80, 96)):
    """Uneven batch of closed meshes: each mesh is a torus grid with
    V ~ logU[1e3, 2e5] (n2 = round(sqrt(V/2)), n1 = 2 n2) or a chain of g tori
    (g ~ U{2..10}, spacing 1.6) extracted on an n^3 grid fitted per axis, n
    drawn from ``pretzel_grids``; type ~ Bernoulli(1/2).  The chain surfaces
    for each (g, n) are extracted once and shared; every mesh gets its own
    N(0,1e-4) jitter and seed vertex from stream base_seed + i."""
    rng = np.random.default_rng(base_seed)
    kinds = rng.integers(0, 2, size=n)
    cache = {}
    out = []
    for i in range(n):
        if kinds[i] == 0:
            V = float(np.exp(rng.uniform(np.log(1e3), np.log(2e5))))
            n2 = max(4, int(round(np.sqrt(V / 2.0))))
            m = torus_grid(2 * n2, n2, 1.0, 0.4, 1e-3, rng_seed=base_seed + i)
        else:
            g = int(rng.integers(2, 11))
            gn = int(pretzel_grids[int(rng.integers(len(pretzel_grids)))])
            if (g, gn) not in cache:
                cache[(g, gn)] = multi_torus(g, gn, sigma=0.0, rng_seed=0)
            base = cache[(g, gn)]
            m = jittered(base, 1e-4, base_seed + i, f"torus_chain{g}_{gn}")
        out.append(m)
    return out


# ---------------------------------------------------------------------------
# large surfaces: marching tetrahedra streamed by slabs of grid planes
# ---------------------------------------------------------------------------
def marching_tets_slabs(plane_f, lo, hi, shape, slab: int = 16, chunk_cells: int = 1 << 21,
                        progress=None) -> Mesh:
    """Level-0 surface of a field given plane by plane: ``plane_f(x, Y, Z)``
    returns f on the grid plane at abscissa x (Y, Z: 2-D coordinate arrays).
    Same extraction as ``marching_tets`` (six tetrahedra per cell, inside
    means f < 0, vertices on crossed tet edges welded by grid-edge key and
    numbered in ascending key order), but only ``slab`` + 1 planes of samples
    are held at a time, so grids of 1024^3 samples fit in host memory."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    nx, ny, nz = (int(s) for s in shape)
    npts = nx * ny * nz
    h = (hi - lo) / (np.array([nx, ny, nz], dtype=np.float64) - 1.0)
    xs = lo[0] + h[0] * np.arange(nx)
    ys = lo[1] + h[1] * np.arange(ny)
    zs = lo[2] + h[2] * np.arange(nz)
    Y, Z = np.meshgrid(ys, zs, indexing="ij")
    corner_off = np.array([dx * ny * nz + dy * nz + dz
                           for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)], dtype=np.int64)
    keys_u, xyz_u, tri_keys = [], [], []
    prev = None                                    # last plane of the previous slab
    for i0 in range(0, nx - 1, slab):
        if progress is not None and i0 % (slab * 16) == 0:
            progress(f"extraction: plane {i0} of {nx}")
        i1 = min(nx - 1, i0 + slab)                # cells i0..i1-1, planes i0..i1
        planes = [prev if (prev is not None and i == i0) else plane_f(xs[i], Y, Z) for i in range(i0, i1 + 1)]
        F = np.stack(planes)
        prev = planes[-1]
        del planes
        neg = F < 0
        nxs = i1 - i0 + 1
        anyin = np.zeros((nxs - 1, ny - 1, nz - 1), dtype=bool)
        allin = np.ones((nxs - 1, ny - 1, nz - 1), dtype=bool)
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    s = neg[dx:nxs - 1 + dx, dy:ny - 1 + dy, dz:nz - 1 + dz]
                    anyin |= s
                    allin &= s
        cells = np.flatnonzero(anyin & ~allin)
        del anyin, allin
        if cells.size == 0:
            continue
        ci, rem = np.divmod(cells, (ny - 1) * (nz - 1))
        cj, ck = np.divmod(rem, nz - 1)
        lbase = ci * ny * nz + cj * nz + ck        # local grid id (slab planes)
        off0 = i0 * ny * nz                        # local -> global grid id
        Ff = F.ravel()
        negf = neg.ravel()
        kl = []
        for s0 in range(0, lbase.size, chunk_cells):
            b = lbase[s0:s0 + chunk_cells]
            for t in range(6):
                g = b[:, None] + corner_off[_TETS[t]][None, :]
                ins = negf[g]
                case = ins[:, 0] * 1 + ins[:, 1] * 2 + ins[:, 2] * 4 + ins[:, 3] * 8
                for k in (0, 1):
                    sel = _NTRI[case] > k
                    if not np.any(sel):
                        continue
                    e = _CASES[case[sel], k]
                    gs = g[sel]
                    ga = np.take_along_axis(gs, e[:, :, 0], axis=1)
                    gb = np.take_along_axis(gs, e[:, :, 1], axis=1)
                    kl.append(np.minimum(ga, gb) * (nxs * ny * nz) + np.maximum(ga, gb))
        lk = np.concatenate(kl, axis=0)
        del kl
        nloc = nxs * ny * nz
        uk, inv = np.unique(lk.ravel(), return_inverse=True)
        ga = uk // nloc
        gb = uk % nloc
        fa = Ff[ga]
        fb = Ff[gb]
        tt = fa / (fa - fb)

        def coords(gid):
            i, r = np.divmod(gid, ny * nz)
            j, kk = np.divmod(r, nz)
            return np.stack([xs[i + i0], ys[j], zs[kk]], axis=1)
        pa = coords(ga)
        pb = coords(gb)
        xyz_u.append(pa + tt[:, None] * (pb - pa))
        gk = (ga + off0) * npts + (gb + off0)      # global edge keys
        keys_u.append(gk)
        tri_keys.append(gk[inv].reshape(-1, 3))
        del F, neg, lk, uk, inv
    allk = np.concatenate(keys_u)
    allx = np.concatenate(xyz_u)
    del keys_u, xyz_u
    u, first = np.unique(allk, return_index=True)
    xyz = allx[first]
    del allk, allx
    tri = np.concatenate([np.searchsorted(u, tk).astype(np.int32) for tk in tri_keys])
    return Mesh(xyz.astype(np.float64), tri, 0, "mt_slabs")


def lattice_plane_sdf(n_cells: int, radius: float):
    """Signed distance to the struts of the cubic lattice with nodes at the
    integer points of [0, n]^3 and a strut of the given radius on every
    edge between neighbouring nodes, evaluated on a plane of constant x:
    for each axis the nearest parallel strut line is found by rounding the
    two other coordinates into [0, n]; beyond the lattice the distance
    along the line is measured to the strut's end."""
    n = float(n_cells)

    def f(x, Y, Z):
        jj = np.clip(np.rint(Y), 0.0, n)
        kk = np.clip(np.rint(Z), 0.0, n)
        ii = min(max(float(np.rint(x)), 0.0), n)
        ex = max(0.0, -x, x - n)
        ey = np.maximum(0.0, np.maximum(-Y, Y - n))
        ez = np.maximum(0.0, np.maximum(-Z, Z - n))
        dyj = Y - jj
        dzk = Z - kk
        dxi = x - ii
        d1 = np.sqrt(dyj * dyj + dzk * dzk + ex * ex)
        d2 = np.sqrt(dxi * dxi + dzk * dzk + ey * ey)
        d3 = np.sqrt(dxi * dxi + dyj * dyj + ez * ez)
        return np.minimum(np.minimum(d1, d2), d3) - radius
    return f


def lattice_genus(n_cells: int) -> int:
    """Genus of the thickened cubic lattice graph: edges - nodes + 1."""
    n = n_cells
    return 3 * n * (n + 1) ** 2 - (n + 1) ** 3 + 1


_MT_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mt_lattice.c")
_MT_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_mt_lattice.so")
_mt = None


def build(force: bool = True) -> str:
    """Compile the C twin of the lattice extraction (gcc, OpenMP, no
    contraction)."""
    if force or not os.path.exists(_MT_LIB) or os.path.getmtime(_MT_LIB) < os.path.getmtime(_MT_SRC):
        tmp = _MT_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99",
                               "-shared", "-fPIC", "-o", tmp, _MT_SRC, "-lm"])
        os.replace(tmp, _MT_LIB)
    return _MT_LIB


def _mt_load():
    global _mt
    if _mt is None:
        build(force=False)
        lib = ctypes.CDLL(_MT_LIB)
        P = ctypes.c_void_p
        lib.mt_lattice.restype = ctypes.c_int
        lib.mt_lattice.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                   P, P, P, P, P, P, P, ctypes.POINTER(P), ctypes.POINTER(P)]
        lib.mt_free.restype = None
        lib.mt_free.argtypes = [P]
        _mt = lib
    return _mt


def lattice_mt_compiled(n_cells: int, radius: float, lo, hi, shape) -> Mesh:
    """The same extraction as ``marching_tets_slabs(lattice_plane_sdf(...))``
    run by the compiled twin in mt_lattice.c: bit-identical vertex positions
    and numbering, the same triangles (in another order), in parallel."""
    lib = _mt_load()
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    tets = np.ascontiguousarray(_TETS, dtype=np.int64)
    cases = np.ascontiguousarray(_CASES, dtype=np.int64)
    ntri = np.ascontiguousarray(_NTRI, dtype=np.int64)
    nv, nf = ctypes.c_int64(), ctypes.c_int64()
    px, pt = ctypes.c_void_p(), ctypes.c_void_p()
    rc = lib.mt_lattice(int(n_cells), float(radius), int(shape[0]), int(shape[1]), int(shape[2]),
                        lo.ctypes.data, hi.ctypes.data, tets.ctypes.data, cases.ctypes.data, ntri.ctypes.data,
                        ctypes.byref(nv), ctypes.byref(nf), ctypes.byref(px), ctypes.byref(pt))
    if rc != 0:
        raise MemoryError("mt_lattice: out of memory")
    try:
        xyz = np.ctypeslib.as_array((ctypes.c_double * (3 * nv.value)).from_address(px.value)).reshape(-1, 3).copy()
        tri = np.ctypeslib.as_array((ctypes.c_int32 * (3 * nf.value)).from_address(pt.value)).reshape(-1, 3).copy()
    finally:
        lib.mt_free(px)
        lib.mt_free(pt)
    return Mesh(xyz, tri, 0, "mt_lattice")


def lattice(n_cells: int = 10, grid: int = 1024, radius: float = 0.15, sigma: float = 0.0,
            rng_seed: int = 0, slab: int = 16, progress=None, compiled: bool = True) -> Mesh:
    """Strut lattice surface: level 0 of ``lattice_plane_sdf`` on grid^3
    samples over [-0.5, n + 0.5]^3, optional N(0, sigma^2) jitter, then a
    random seed vertex from rng_seed.  Genus ``lattice_genus(n_cells)``.
    compiled=True extracts with the C twin (same vertices and triangles,
    triangles in another order), else with the numpy slab extraction."""
    lo = (-0.5, -0.5, -0.5)
    hi = (n_cells + 0.5,) * 3
    if compiled:
        m = lattice_mt_compiled(n_cells, radius, lo, hi, (grid, grid, grid))
    else:
        m = marching_tets_slabs(lattice_plane_sdf(n_cells, radius), lo, hi, (grid, grid, grid), slab,
                                progress=progress)
    m = jittered(m, sigma, rng_seed, f"lattice{n_cells}_{grid}") if sigma > 0 else \
        Mesh(m.xyz, m.tri, 0, f"lattice{n_cells}_{grid}")
    return m if sigma > 0 else pick_seed(m, rng_seed)


# ---------------------------------------------------------------------------
# unjittered voxel surfaces and the 7-vertex torus
# ---------------------------------------------------------------------------
def voxel_surface(occ, center: bool = True, name: str = "voxel") -> Mesh:
    """Boundary of a set of unit voxels: occ[i, j, k] True fills the cube
    [i, i+1] x [j, j+1] x [k, k+1].  Each exposed unit face becomes four
    triangles around its centre (center=True: the face's full symmetry is
    kept) or two triangles split along the diagonal on which both in-plane
    coordinates increase (a choice every permutation of the axes maps to
    itself).  Triangles are counter-clockwise seen from outside; vertices are
    welded by their doubled integer coordinates and numbered in ascending
    (x, y, z) order.  No jitter; seed vertex 0.  Voxels that touch only along
    an edge or at a corner make a non-manifold surface: the shapes used here
    have none."""
    occ = np.asarray(occ, dtype=bool)
    P = np.pad(occ, 1)
    quads = []
    for ax in range(3):
        a1, a2 = (ax + 1) % 3, (ax + 2) % 3
        e1 = np.zeros(3, np.int64)
        e1[a1] = 1
        e2 = np.zeros(3, np.int64)
        e2[a2] = 1
        for sgn in (1, -1):
            face = P & ~np.roll(P, -sgn, axis=ax)       # filled voxel, empty neighbour
            idx = np.argwhere(face).astype(np.int64) - 1
            if idx.size == 0:
                continue
            base = idx.copy()
            if sgn == 1:
                base[:, ax] += 1
            p0, p1, p2, p3 = base, base + e1, base + e1 + e2, base + e2
            # (e1, e2, e_ax) is right-handed: p0 p1 p2 p3 is counter-clockwise seen from +ax
            quads.append(np.stack([p0, p1, p2, p3] if sgn == 1 else [p0, p3, p2, p1], axis=1))
    Q = 2 * np.concatenate(quads)                        # [nq, 4, 3] doubled coordinates
    if center:
        cen = Q.sum(axis=1) // 4
        T = np.concatenate([np.stack([Q[:, k], Q[:, (k + 1) % 4], cen], axis=1) for k in range(4)])
    else:
        lo = np.argmin(Q.sum(axis=2), axis=1)            # corner with the smallest coordinate sum
        r = np.arange(Q.shape[0])
        c = [Q[r, (lo + k) % 4] for k in range(4)]
        T = np.concatenate([np.stack([c[0], c[1], c[2]], axis=1), np.stack([c[0], c[2], c[3]], axis=1)])
    flat = T.reshape(-1, 3)
    M = int(flat.max()) + 1
    key = (flat[:, 0] * M + flat[:, 1]) * M + flat[:, 2]
    uk, inv = np.unique(key, return_inverse=True)
    xyz = np.stack([uk // (M * M), (uk // M) % M, uk % M], axis=1).astype(np.float64) / 2.0
    return Mesh(xyz, inv.reshape(-1, 3).astype(np.int32), 0, name)


def voxel_frame(n_cells: int = 1, length: int = 2, bar: int = 1, center: bool = True) -> Mesh:
    """Voxel jungle gym: bars of bar x bar voxels along every edge of an
    n_cells^3 cubic lattice with `length` empty voxels between bars (a voxel
    is filled when at least two of its three coordinates fall in a bar
    interval).  Genus = struts - nodes + 1, as for the strut lattice."""
    N = n_cells * (length + bar) + bar
    r = (np.arange(N) % (length + bar)) < bar
    I, J, K = np.meshgrid(r, r, r, indexing="ij")
    occ = (I.astype(np.int64) + J + K) >= 2
    return voxel_surface(occ, center, f"voxel_frame{n_cells}_{length}_{bar}{'c' if center else 'd'}")


def csaszar_torus() -> Mesh:
    """The 7-vertex torus: triangles (i, i+1, i+3) and (i, i+3, i+2) mod 7,
    vertices on a twisted ring (the coordinates only matter for lengths and
    positions; the triangulation is what the method sees)."""
    t = []
    for i in range(7):
        t.append((i, (i + 1) % 7, (i + 3) % 7))
        t.append((i, (i + 3) % 7, (i + 2) % 7))
    ang = np.arange(7) * 2.0 * np.pi / 7.0
    xyz = np.stack([np.cos(ang), np.sin(ang), 0.3 * np.cos(3.0 * ang)], axis=1)
    return Mesh(xyz.astype(np.float64), np.array(t, dtype=np.int32), 0, "csaszar7")
