"""Seeded synthetic scenes shaped like the paper's workloads.

Every array is produced with ``numpy.random.default_rng(seed)`` and returned in
the layout the library and the oracle both read:

* ``vtx``      float32 [V, 3]   vertex coordinates in metres
* ``tri``      int32   [M, 3]   vertex indices of each flat triangle
* ``material`` int32   [M]      material index per triangle
* ``plane_id`` int32   [M]      coplanar-group id per triangle (0 <= id < M)
* ``alpha``    float32 [n_mat, 8] absorption per material and octave band
* ``beta``     float32 [8]      air absorption per band, energy, 1/m
* ``src``      float32 [3]      point source
* ``rcv``      float32 [n_rcv, 4] receiver spheres (x, y, z, r)

Octave bands are 62.5 Hz ... 8 kHz (Table 1 of the paper).  The absorption rows
printed in Table 1 are read from ``tests/golden/table1_absorption.txt``-equivalent
constants below.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BAND_CENTRES = np.array([62.5 * 2.0 ** b for b in range(8)])  # Hz, Table 1 columns

# Table 1 of the paper: Odeon rows (reference number -> 8-band absorption).
TABLE1 = {
    1: [1, 1, 1, 1, 1, 1, 1, 1],                                  # 100 % absorbent
    2: [0, 0, 0, 0, 0, 0, 0, 0],                                  # 100 % reflecting
    107: [0.36, 0.36, 0.44, 0.31, 0.29, 0.39, 0.25, 0.25],        # concrete block, coarse
    3000: [0.4, 0.4, 0.3, 0.2, 0.17, 0.15, 0.1, 0.1],             # hollow wooden podium
}


@dataclasses.dataclass
class Scene:
    name: str
    vtx: np.ndarray
    tri: np.ndarray
    material: np.ndarray
    plane_id: np.ndarray
    alpha: np.ndarray
    closed: bool
    src: np.ndarray = None
    rcv: np.ndarray = None
    beta: np.ndarray = None
    n_rays: int = 0
    max_reflections: int = 0
    c: float = 343.0
    fs: float = 48000.0
    ir_seconds: float = 0.0

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_vtx(self) -> int:
        return int(self.vtx.shape[0])

    @property
    def n_mat(self) -> int:
        return int(self.alpha.shape[0])

    @property
    def ir_len(self) -> int:
        return int(round(self.fs * self.ir_seconds))

    @property
    def max_path_length(self) -> float:
        """c*T plus the largest receiver radius (rays stop once past it)."""
        rmax = float(self.rcv[:, 3].max()) if self.rcv is not None and len(self.rcv) else 0.0
        return float(self.c * self.ir_seconds + rmax)

    def diag(self) -> float:
        v = self.vtx.astype(np.float64)
        return float(np.linalg.norm(v.max(0) - v.min(0)))


# ----------------------------------------------------------------------------
# mesh helpers (pure bookkeeping: vertex lattices and index lists)
# ----------------------------------------------------------------------------

def _quads_to_tris(q: np.ndarray) -> np.ndarray:
    """(a,b,c,d) cyclic quads -> triangles (a,b,c), (a,c,d): fixed diagonal a-c."""
    t1 = q[:, [0, 1, 2]]
    t2 = q[:, [0, 2, 3]]
    return np.stack([t1, t2], axis=1).reshape(-1, 3)


def _grid_quads(idx: np.ndarray) -> np.ndarray:
    """Quads of a 2-D vertex-index grid idx[i, j] (cells between neighbours)."""
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    return np.stack([a, b, c, d], axis=1)


def edge_use_counts(tri: np.ndarray) -> np.ndarray:
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    _, counts = np.unique(e, axis=0, return_counts=True)
    return counts


def is_watertight(tri: np.ndarray) -> bool:
    """Every undirected edge is shared by exactly two triangles."""
    return bool(np.all(edge_use_counts(tri) == 2))


def _tri_areas(vtx: np.ndarray, tri: np.ndarray) -> np.ndarray:
    v = vtx.astype(np.float64)
    e1 = v[tri[:, 1]] - v[tri[:, 0]]
    e2 = v[tri[:, 2]] - v[tri[:, 0]]
    return 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)


def _check(scene: Scene, expect_tris: Optional[int] = None) -> Scene:
    assert scene.vtx.dtype == np.float32 and scene.tri.dtype == np.int32
    assert scene.material.dtype == np.int32 and scene.plane_id.dtype == np.int32
    assert np.all(np.isfinite(scene.vtx))
    assert scene.tri.min() >= 0 and scene.tri.max() < scene.n_vtx
    assert np.all(_tri_areas(scene.vtx, scene.tri) > 0), "zero-area triangle"
    assert scene.plane_id.min() >= 0 and scene.plane_id.max() < scene.n_tri
    assert scene.material.min() >= 0 and scene.material.max() < scene.n_mat
    if expect_tris is not None:
        assert scene.n_tri == expect_tris, (scene.name, scene.n_tri, expect_tris)
    if scene.closed:
        assert is_watertight(scene.tri), scene.name
    return scene


def _truncated_normal(rng: np.random.Generator, shape, sigma: float, cut: float = 3.0):
    x = rng.standard_normal(shape)
    bad = np.abs(x) > cut
    while bad.any():
        x[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(x) > cut
    return x * sigma


# ----------------------------------------------------------------------------
# box rooms
# ----------------------------------------------------------------------------

def box_mesh(dims, n=(1, 1, 1), jitter_sigma: float = 0.0, rng=None,
             plane_per_wall: bool = True):
    """Closed box [0,Lx]x[0,Ly]x[0,Lz] as shared-vertex grids on its six walls.

    Walls (material index = wall index): 0 x=0, 1 x=Lx, 2 y=0, 3 y=Ly, 4 z=0,
    5 z=Lz.  With n=(1,1,1) this is the 8-vertex, 12-triangle shoebox.
    """
    nx, ny, nz = n
    Lx, Ly, Lz = dims
    I, J, K = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    boundary = (I == 0) | (I == nx) | (J == 0) | (J == ny) | (K == 0) | (K == nz)
    idx = -np.ones(I.shape, dtype=np.int64)
    idx[boundary] = np.arange(int(boundary.sum()))
    pts = np.stack([I[boundary] * (Lx / nx), J[boundary] * (Ly / ny), K[boundary] * (Lz / nz)],
                   axis=1).astype(np.float64)
    # exact wall coordinates for the far walls (avoid i*(L/n) rounding)
    pts[I[boundary] == nx, 0] = Lx
    pts[J[boundary] == ny, 1] = Ly
    pts[K[boundary] == nz, 2] = Lz
    if jitter_sigma > 0:
        pts = pts + _truncated_normal(rng, pts.shape, jitter_sigma)
    walls = [
        idx[0, :, :], idx[nx, :, :].T,       # x = 0, x = Lx  (orientation irrelevant)
        idx[:, 0, :].T, idx[:, ny, :],
        idx[:, :, 0], idx[:, :, nz].T,
    ]
    tris, mats = [], []
    for w, g in enumerate(walls):
        t = _quads_to_tris(_grid_quads(g))
        tris.append(t)
        mats.append(np.full(len(t), w, dtype=np.int32))
    tri = np.concatenate(tris).astype(np.int32)
    mat = np.concatenate(mats)
    if plane_per_wall:
        # plane id = lowest triangle index of each wall (the group's representative)
        first = np.concatenate([[0], np.cumsum([len(t) for t in tris])[:-1]])
        plane = first[mat].astype(np.int32)
    else:
        plane = np.arange(len(tri), dtype=np.int32)
    return pts.astype(np.float32), tri, mat, plane


def random_alpha(rng, n_mat: int, lo=0.02, hi=0.3) -> np.ndarray:
    return rng.uniform(lo, hi, size=(n_mat, 8)).astype(np.float32)


def shoebox_c1(seed: int = 1) -> Scene:
    """10 x 7 x 3 m shoebox as 12 triangles; one receiver (r = 0.3 m)."""
    rng = np.random.default_rng(seed)
    vtx, tri, mat, plane = box_mesh((10.0, 7.0, 3.0))
    alpha = random_alpha(rng, 6)
    s = Scene("C1 shoebox 12 tris", vtx, tri, mat, plane, alpha, closed=True,
              src=np.array([3.17, 2.41, 1.63], np.float32),
              rcv=np.array([[7.29, 4.87, 1.38, 0.3]], np.float32),
              beta=np.zeros(8, np.float32), n_rays=10_000, max_reflections=20,
              ir_seconds=0.5)
    return _check(s, 12)


def paper_box(seed: int = 11, n_rays: int = 100_000, max_reflections: int = 6) -> Scene:
    """The paper's [5,4,3] m validation box: 12 triangles, source [4,2,1.7],
    receiver [2,2,1.7] with r = 0.2 m (shoe-box comparison section)."""
    rng = np.random.default_rng(seed)
    vtx, tri, mat, plane = box_mesh((5.0, 4.0, 3.0))
    alpha = random_alpha(rng, 6)
    s = Scene("paper box 5x4x3", vtx, tri, mat, plane, alpha, closed=True,
              src=np.array([4.0, 2.0, 1.7], np.float32),
              rcv=np.array([[2.0, 2.0, 1.7, 0.2]], np.float32),
              beta=iso9613_beta(), n_rays=n_rays, max_reflections=max_reflections,
              ir_seconds=0.25)
    return _check(s, 12)


def tessellated_box_c2(seed: int = 2, jitter: bool = True) -> Scene:
    """The C1 box as 144x101x43 shared-vertex grids: 100,316 triangles, 50,160
    vertices.  Jittered variant: truncated-Gaussian sigma = 1 cm on every shared
    vertex (watertight), plane id = triangle id.  Flat variant: plane id = wall."""
    rng = np.random.default_rng(seed)
    vtx, tri, mat, plane = box_mesh((10.0, 7.0, 3.0), (144, 101, 43),
                                    jitter_sigma=0.01 if jitter else 0.0, rng=rng,
                                    plane_per_wall=not jitter)
    assert vtx.shape[0] == 50_160
    alpha = random_alpha(rng, 6)
    rcv = np.concatenate([rng.uniform([1, 1, 0.8], [9, 6, 2.2], size=(3, 3)),
                          np.full((3, 1), 0.3)], axis=1).astype(np.float32)
    s = Scene("C2 tessellated box 100k" + (" jittered" if jitter else " flat"),
              vtx, tri, mat, plane, alpha, closed=True,
              src=np.array([3.17, 2.41, 1.63], np.float32), rcv=rcv,
              beta=iso9613_beta(), n_rays=1_000_000, max_reflections=50, ir_seconds=1.0)
    return _check(s, 100_316)


# ----------------------------------------------------------------------------
# open-air theater (stand-in for the 436k-face Orange mesh)
# ----------------------------------------------------------------------------

class _MeshBuilder:
    def __init__(self):
        self.v: List[np.ndarray] = []
        self.t: List[np.ndarray] = []
        self.m: List[np.ndarray] = []
        self.p: List[np.ndarray] = []   # -1 => plane id = own triangle id
        self.nv = 0
        self.nt = 0
        self.groups = 0

    def add(self, verts, tris, material: int, coplanar: bool):
        verts = np.asarray(verts, np.float64).reshape(-1, 3)
        tris = np.asarray(tris, np.int64).reshape(-1, 3) + self.nv
        self.v.append(verts)
        self.t.append(tris)
        self.m.append(np.full(len(tris), material, np.int32))
        if coplanar:
            self.p.append(np.full(len(tris), self.nt, np.int64))   # representative = first tri
        else:
            self.p.append(self.nt + np.arange(len(tris)))
        self.nv += len(verts)
        self.nt += len(tris)

    def grid(self, pts2d: np.ndarray, material: int, coplanar: bool):
        """pts2d: [a, b, 3] vertex grid -> quads -> triangles."""
        a, b, _ = pts2d.shape
        idx = np.arange(a * b).reshape(a, b)
        self.add(pts2d.reshape(-1, 3), _quads_to_tris(_grid_quads(idx)), material, coplanar)

    def finish(self):
        vtx = np.concatenate(self.v).astype(np.float32)
        tri = np.concatenate(self.t).astype(np.int32)
        mat = np.concatenate(self.m)
        plane = np.concatenate(self.p).astype(np.int32)
        return vtx, tri, mat, plane


THEATER_STAGE_Z = 1.0
THEATER_RISER = 0.55
THEATER_TREAD = 0.95


def _tier_height(t: int) -> float:
    return THEATER_RISER * (t + 1)


def _tier_radius(t: int) -> float:
    return 12.0 + THEATER_TREAD * t


def theater_c3(seed: int = 3, n_rays: int = 1_000_000, max_reflections: int = 60,
               ir_seconds: float = 2.0) -> Scene:
    """Synthetic open-air theater of 436,120 triangles (no ceiling).

    * orchestra: half annulus r in [1, 12] m at z = 0, 1024 x 10 cells (20,480)
    * cavea: 40 tiers from r = 12 to 50 m, riser 0.55 m, tread 0.95 m, each a
      riser strip and a tread strip over the semicircle y >= 0 with 1024 angular
      cells (163,840)
    * stage floor 100 x 30 m at z = 1 (6,000) and its 1 m front riser (200)
    * stage wall 100 x 35 m at y = -30 as a 440 x 200 grid with seeded smooth
      displacement noise of 0.4 m amplitude, standing for ornaments (176,000)
    * 200 columns (4 stories x 50), 16-gon, 10 height segments with slight
      entasis (64,000) plus 16-gon fan caps (5,600)

    Materials: 0 = concrete block, coarse (Table 1 ref 107) everywhere except
    1 = hollow wooden podium (Table 1 ref 3000) on the stage floor.  Flat groups
    (orchestra, each tread, stage floor, stage front, each column cap) share one
    plane id; curved or displaced surfaces use one plane id per triangle.
    """
    rng = np.random.default_rng(seed)
    mb = _MeshBuilder()
    nseg = 1024
    th = np.linspace(0.0, math.pi, nseg + 1)
    cth, sth = np.cos(th), np.sin(th)

    def ring(r, z):
        return np.stack([r * cth, r * sth, np.full_like(th, z)], axis=1)

    # orchestra
    radii = np.linspace(1.0, 12.0, 11)
    g = np.stack([ring(r, 0.0) for r in radii], axis=0)
    mb.grid(g, 0, coplanar=True)
    # cavea: alternating riser / tread strips sharing rings
    z_prev = 0.0
    for t in range(40):
        r_in, r_out, z_t = _tier_radius(t), _tier_radius(t) + THEATER_TREAD, _tier_height(t)
        mb.grid(np.stack([ring(r_in, z_prev), ring(r_in, z_t)], axis=0), 0, coplanar=False)
        mb.grid(np.stack([ring(r_in, z_t), ring(r_out, z_t)], axis=0), 0, coplanar=True)
        z_prev = z_t
    # stage floor and its front riser
    xs = np.linspace(-50.0, 50.0, 101)
    ys = np.linspace(-30.0, 0.0, 31)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    mb.grid(np.stack([X, Y, np.full_like(X, THEATER_STAGE_Z)], axis=2), 1, coplanar=True)
    X, Z = np.meshgrid(xs, np.array([0.0, THEATER_STAGE_Z]), indexing="ij")
    mb.grid(np.stack([X, np.zeros_like(X), Z], axis=2), 0, coplanar=True)
    # stage wall with smooth displacement noise
    xw = np.linspace(-50.0, 50.0, 441)
    zw = np.linspace(THEATER_STAGE_Z, THEATER_STAGE_Z + 35.0, 201)
    X, Z = np.meshgrid(xw, zw, indexing="ij")
    disp = np.zeros_like(X)
    for _ in range(12):
        kx, kz = rng.uniform(0.2, 2.5, size=2)
        ph = rng.uniform(0, 2 * math.pi, size=2)
        disp += np.sin(kx * X + ph[0]) * np.sin(kz * Z + ph[1])
    disp *= 0.4 / np.abs(disp).max()
    mb.grid(np.stack([X, -30.0 + disp, Z], axis=2), 0, coplanar=False)
    # columns: 4 stories x 50, 16-gon, 10 segments, entasis, fan caps
    nside, nh, r0, hcol = 16, 10, 0.35, 8.0
    ang = np.arange(nside) * (2 * math.pi / nside)
    for story in range(4):
        z0 = THEATER_STAGE_Z + 8.75 * story + 0.4
        for i in range(50):
            cx, cy = -49.0 + 2.0 * i, -28.5
            hs = np.linspace(0.0, hcol, nh + 1)
            rr = r0 * (1.0 + 0.04 * np.sin(math.pi * hs / hcol)) * (1.0 - 0.08 * hs / hcol)
            pts = np.stack([
                np.stack([cx + rr[k] * np.cos(ang), cy + rr[k] * np.sin(ang),
                          np.full(nside, z0 + hs[k])], axis=1) for k in range(nh + 1)])
            # side: rings x (sides + wrap) grid
            wrap = np.concatenate([pts, pts[:, :1]], axis=1)            # [11, 17, 3]
            mb.grid(wrap, 0, coplanar=False)
            for k, flip in ((0, True), (nh, False)):
                cap = pts[k]
                fan = np.array([[0, j, j + 1] for j in range(1, nside - 1)])
                if flip:
                    fan = fan[:, [0, 2, 1]]
                mb.add(cap, fan, 0, coplanar=True)
    vtx, tri, mat, plane = mb.finish()
    alpha = np.array([TABLE1[107], TABLE1[3000]], np.float32)
    axis = math.pi / 2
    spots = [(2, axis), (8, axis), (16, axis), (26, axis), (36, axis),
             (10, axis - math.pi / 4), (20, axis + math.pi / 4), (30, axis + 75 * math.pi / 180)]
    rcv = []
    for t, a in spots:
        r = _tier_radius(t) + 0.5 * THEATER_TREAD
        rcv.append([r * math.cos(a), r * math.sin(a), _tier_height(t) + 1.2, 2.0])
    s = Scene("C3 open-air theater 436k", vtx, tri, mat, plane, alpha, closed=False,
              src=np.array([0.0, -1.0, THEATER_STAGE_Z + 1.6], np.float32),
              rcv=np.array(rcv, np.float32), beta=iso9613_beta(), n_rays=n_rays,
              max_reflections=max_reflections, ir_seconds=ir_seconds)
    return _check(s, 436_120)


# ----------------------------------------------------------------------------
# small test geometries
# ----------------------------------------------------------------------------

def icosphere(level: int, radius: float = 1.0):
    """Unit icosphere: 20 * 4**level faces, vertices projected to the sphere."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    faces = f
    for _ in range(level):
        cache = {}
        new_faces = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    vtx = (np.array(verts) * radius).astype(np.float32)
    tri = np.array(faces, np.int32)
    return vtx, tri


def sphere_room(level: int = 4) -> Scene:
    """100 % reflecting unit sphere, source and receiver at the centre."""
    vtx, tri = icosphere(level)
    m = len(tri)
    s = Scene(f"unit icosphere {m}", vtx, tri, np.zeros(m, np.int32), np.arange(m, dtype=np.int32),
              np.zeros((1, 8), np.float32), closed=True,
              src=np.zeros(3, np.float32), rcv=np.array([[0, 0, 0, 0.05]], np.float32),
              beta=np.zeros(8, np.float32), n_rays=10_000, max_reflections=6, ir_seconds=0.05)
    return _check(s, 20 * 4 ** level)


def open_scene_far_triangle() -> Scene:
    """A single far-away triangle: every ray from the origin region escapes
    except those aimed at it; used for the free-field (1/d^2) law."""
    vtx = np.array([[1000, 1000, 1000], [1001, 1000, 1000], [1000, 1001, 1000]], np.float32)
    tri = np.array([[0, 1, 2]], np.int32)
    return _check(Scene("open far triangle", vtx, tri, np.zeros(1, np.int32), np.zeros(1, np.int32),
                        np.zeros((1, 8), np.float32), closed=False, beta=np.zeros(8, np.float32)))


def lroom(seed: int = 5, dims=(8.0, 6.0, 3.0), notch=(4.0, 3.0)):
    """Closed L-shaped room: a box with one corner block removed, as 12 quads
    on its faces (the floor and ceiling L-polygons split into three rectangles
    so every edge stays shared).  Returns (vtx, tri, material, plane)."""
    Lx, Ly, Lz = dims
    nx, ny = notch
    xs = [0.0, nx, Lx]
    ys = [0.0, ny, Ly]
    # L = all cells of the 2x2 footprint grid except (1,1) (x>nx, y>ny)
    cells = [(0, 0), (1, 0), (0, 1)]
    vid = {}
    verts = []

    def v(ix, iy, iz):
        key = (ix, iy, iz)
        if key not in vid:
            vid[key] = len(verts)
            verts.append((xs[ix], ys[iy], [0.0, Lz][iz]))
        return vid[key]

    quads, mats = [], []
    for iz, m in ((0, 4), (1, 5)):                       # floor, ceiling
        for cx, cy in cells:
            quads.append((v(cx, cy, iz), v(cx + 1, cy, iz), v(cx + 1, cy + 1, iz), v(cx, cy + 1, iz)))
            mats.append(m)
    # perimeter walls of the L, split at grid lines so edges match the floor split
    boundary = [((0, 0), (1, 0), 2), ((1, 0), (2, 0), 2), ((2, 0), (2, 1), 1), ((2, 1), (1, 1), 3),
                ((1, 1), (1, 2), 1), ((1, 2), (0, 2), 3), ((0, 2), (0, 1), 0), ((0, 1), (0, 0), 0)]
    for (ax, ay), (bx, by), m in boundary:
        quads.append((v(ax, ay, 0), v(bx, by, 0), v(bx, by, 1), v(ax, ay, 1)))
        mats.append(m)
    # the floor/ceiling splits add interior edges on the footprint (0..2 x 0..2 grid):
    # floor cells (0,0),(1,0),(0,1) share edges among themselves -> fine
    q = np.array(quads, np.int64)
    tri = _quads_to_tris(q).astype(np.int32)
    mat = np.repeat(np.array(mats, np.int32), 2)
    # plane ids: group coplanar faces (same axis-aligned plane)
    vv = np.array(verts, np.float64)
    keys = {}
    plane = np.empty(len(tri), np.int32)
    for i, t in enumerate(tri):
        p = vv[t]
        for ax in range(3):
            if np.all(p[:, ax] == p[0, ax]):
                key = (ax, p[0, ax])
                break
        if key not in keys:
            keys[key] = i
        plane[i] = keys[key]
    return np.array(verts, np.float32), tri, mat, plane


def tetra_room(scale: float = 4.0):
    """Closed regular-ish tetrahedron room (4 triangles, 4 planes)."""
    v = np.array([[0, 0, 0], [1, 0, 0], [0.5, math.sqrt(3) / 2, 0],
                  [0.5, math.sqrt(3) / 6, math.sqrt(2.0 / 3.0)]], np.float64) * scale
    tri = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [2, 0, 3]], np.int32)
    return v.astype(np.float32), tri, np.arange(4, dtype=np.int32), np.arange(4, dtype=np.int32)


def tessellated_tetra(k: int, n_rays: int = 0) -> Scene:
    """Regular tetrahedron inscribed in the unit sphere, each face a
    triangular grid of k^2 triangles (4 k^2 in all), source at the centre:
    the workload of the paper's complexity study (one iteration with N rays
    and M faces, "Tree-base acceleration", Table 2).  Grid points are built
    from integer barycentric coordinates on the tetrahedron's 4 vertices, so
    points on shared edges are the same vertex for both faces (watertight).
    Each face is one material; each triangle is its own plane id (the FP32
    vertices of a tilted face are not coplanar to 1e-9 of the diagonal)."""
    A = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float64) / math.sqrt(3.0)
    faces = [(0, 2, 1), (0, 1, 3), (1, 2, 3), (2, 0, 3)]      # outward orientation irrelevant here
    index, verts, tris, mats = {}, [], [], []

    def vid(bary):
        if bary not in index:
            index[bary] = len(verts)
            verts.append(sum(b * A[q] for q, b in enumerate(bary)) / k)
        return index[bary]

    for f, (a, b, c) in enumerate(faces):
        def pt(i, j):
            bary = [0, 0, 0, 0]
            bary[a] += k - i - j
            bary[b] += i
            bary[c] += j
            return vid(tuple(bary))
        for i in range(k):
            for j in range(k - i):
                tris.append((pt(i, j), pt(i + 1, j), pt(i, j + 1)))
                mats.append(f)
                if i + j < k - 1:
                    tris.append((pt(i + 1, j), pt(i + 1, j + 1), pt(i, j + 1)))
                    mats.append(f)
    tri = np.array(tris, np.int32)
    mat = np.array(mats, np.int32)
    plane = np.arange(len(tri), dtype=np.int32)
    s = Scene(f"tetra k={k} {len(tri)} tris", np.array(verts, np.float32), tri, mat, plane,
              np.full((4, 8), 0.1, np.float32), closed=True, src=np.zeros(3, np.float32),
              rcv=np.array([[0.0, 0.0, 0.0, 0.05]], np.float32), beta=np.zeros(8, np.float32),
              n_rays=n_rays or len(tri), max_reflections=0, ir_seconds=0.01)
    return _check(s)


# ----------------------------------------------------------------------------
# batched rooms (many rooms of uneven size)
# ----------------------------------------------------------------------------

def voxel_surface(inside: np.ndarray, spacing):
    """Closed triangle surface of a union of lattice cells.

    inside: bool [nx, ny, nz] (True = air).  Every cell face between an inside
    cell and an outside cell (or the lattice border) becomes two triangles;
    vertices are shared lattice points, so the surface is watertight.  Faces
    in one axis-aligned plane share a plane id (their lowest triangle index);
    material = face orientation: 0 -x, 1 +x, 2 -y, 3 +y, 4 floor, 5 ceiling
    (the direction the wall faces into the room)."""
    nx, ny, nz = inside.shape
    pad = np.zeros((nx + 2, ny + 2, nz + 2), bool)
    pad[1:-1, 1:-1, 1:-1] = inside
    quads, mats, keys = [], [], []
    V = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k   # noqa: E731
    for ax in range(3):
        a_ = np.moveaxis(pad, ax, 0)
        diff = a_[1:].astype(np.int8) - a_[:-1].astype(np.int8)       # [n_ax+1, ., .] face planes
        for sign, mat in ((1, 2 * ax), (-1, 2 * ax + 1)):
            # sign=+1: outside -> inside going +axis: wall faces +axis into the room... material by facing
            f = np.argwhere(diff == sign)
            if len(f) == 0:
                continue
            f[:, 1:] -= 1                                               # back to cell coordinates
            p = f[:, 0]
            u = f[:, 1]
            w = f[:, 2]
            if ax == 0:
                c = [(p, u, w), (p, u + 1, w), (p, u + 1, w + 1), (p, u, w + 1)]
            elif ax == 1:
                c = [(u, p, w), (u + 1, p, w), (u + 1, p, w + 1), (u, p, w + 1)]
            else:
                c = [(u, w, p), (u + 1, w, p), (u + 1, w + 1, p), (u, w + 1, p)]
            q = np.stack([V(*cc) for cc in c], axis=1)
            quads.append(q)
            mats.append(np.full(len(q), mat, np.int32))
            keys.append(np.stack([np.full(len(q), ax), p], axis=1))
    q = np.concatenate(quads)
    mat = np.concatenate(mats)
    key = np.concatenate(keys)
    tri = _quads_to_tris(q)
    mat = np.repeat(mat, 2)
    key = np.repeat(key, 2, axis=0)
    used, inv = np.unique(tri.ravel(), return_inverse=True)
    tri = inv.reshape(-1, 3).astype(np.int32)
    ii = used // ((ny + 1) * (nz + 1))
    jj = (used // (nz + 1)) % (ny + 1)
    kk = used % (nz + 1)
    vtx = np.stack([ii * spacing[0], jj * spacing[1], kk * spacing[2]], axis=1).astype(np.float32)
    # plane ids: lowest triangle index of each (axis, plane index) group
    _, first, grp = np.unique(key, axis=0, return_index=True, return_inverse=True)
    plane = first[grp.ravel()].astype(np.int32)
    return vtx, tri, mat, plane


def _room_cells(kind: int, n):
    nx, ny, nz = n
    inside = np.ones((nx, ny, nz), bool)
    if kind == 1:                                  # L-shape: remove one corner block
        inside[nx // 2:, ny // 2:, :] = False
    elif kind == 2:                                # tiered floor: 3 steps rising along y
        step = max(1, nz // 6)
        for t in range(1, 4):
            inside[:, (t * ny) // 4:, : step * t] = False
    return inside


def _interior_points(rng, inside, spacing, n, margin):
    """Seeded points inside the air cells at least `margin` from any wall."""
    nx, ny, nz = inside.shape
    hi = np.array([nx, ny, nz]) * np.asarray(spacing)
    out = []
    while len(out) < n:
        p = rng.uniform(0, hi)
        ok = True
        for dx in (-margin, 0, margin):
            for dy in (-margin, 0, margin):
                for dz in (-margin, 0, margin):
                    q = p + (dx, dy, dz)
                    c = np.floor(q / spacing).astype(int)
                    if np.any(c < 0) or np.any(c >= (nx, ny, nz)) or not inside[tuple(c)]:
                        ok = False
        if ok:
            out.append(p)
    return np.array(out, np.float32)


def batched_rooms(seed: int = 4, n_rooms: int = 8, pairs_per_room: int = 8,
                  m_lo: float = 1000.0, m_hi: float = 200_000.0, rays_per_pair: int = 200_000,
                  max_reflections: int = 50, ir_seconds: float = 1.0,
                  alpha_range=(0.02, 0.3)) -> List[Scene]:
    """Rooms of uneven size M_i ~ m_lo (m_hi/m_lo)^(i/(n-1)), cycling through
    shoebox, L-shape and tiered floor, dims U[4, 30] m (height <= 12 m), each
    a watertight lattice surface with exact coplanar plane groups; 6
    materials per room (by wall orientation), alpha ~ U[alpha_range];
    pairs_per_room (source, receiver) pairs at least 1 m from the walls,
    receiver radius 0.3 m.  scene.src holds [pairs, 3] sources and scene.rcv
    the [pairs, 4] receivers (pair p = source p with receiver p)."""
    rng = np.random.default_rng(seed)
    rooms = []
    for i in range(n_rooms):
        frac = i / max(1, n_rooms - 1)
        target = m_lo * (m_hi / m_lo) ** frac
        rooms.append(_lattice_room(rng, i, target, i % 3, pairs_per_room, alpha_range, rays_per_pair,
                                   max_reflections, ir_seconds))
    return rooms


def _lattice_room(rng, i, target, kind, pairs, alpha_range, rays, max_reflections, ir_seconds) -> Scene:
    d = rng.uniform(4.0, 30.0, size=3)
    dims = (float(d[0]), float(d[1]), float(min(d[2], 12.0)))
    area = 2 * (dims[0] * dims[1] + dims[1] * dims[2] + dims[0] * dims[2])
    h = math.sqrt(2 * area / target)          # a lattice box surface has 2 area / h^2 triangles
    n = tuple(max(2, int(round(L / h))) for L in dims)
    spacing = tuple(L / k for L, k in zip(dims, n))
    inside = _room_cells(kind, n)
    vtx, tri, mat, plane = voxel_surface(inside, spacing)
    alpha = random_alpha(rng, 6, *alpha_range)
    srcs = _interior_points(rng, inside, spacing, pairs, 1.0)
    rcvs = np.concatenate([_interior_points(rng, inside, spacing, pairs, 1.0),
                           np.full((pairs, 1), 0.3, np.float32)], axis=1).astype(np.float32)
    s = Scene(f"room{i} kind{kind} {len(tri)} tris", vtx, tri, mat, plane, alpha, closed=True,
              src=srcs, rcv=rcvs, beta=iso9613_beta(), n_rays=rays,
              max_reflections=max_reflections, ir_seconds=ir_seconds)
    return _check(s)


def surrogate_rooms(seed: int = 5, n_rooms: int = 2000, m_lo: float = 1000.0, m_hi: float = 50_000.0,
                    alpha_range=(0.02, 0.5), rays_per_pair: int = 100_000, max_reflections: int = 60,
                    ir_seconds: float = 2.0, first: int = 0) -> List[Scene]:
    """Training rooms for the late-tail surrogate: like batched_rooms, but the
    triangle count is log-uniform in [m_lo, m_hi] and the shape (shoebox,
    L-shape, tiered floor) is drawn at random; one (source, receiver) pair
    per room.  Rooms first .. n_rooms-1 of the seeded sequence are returned
    (every room consumes the same generator state as when all are built)."""
    rng = np.random.default_rng(seed)
    rooms = []
    for i in range(n_rooms):
        target = float(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi))))
        kind = int(rng.integers(0, 3))
        sub = np.random.default_rng([seed, i])
        if i >= first:
            rooms.append(_lattice_room(sub, i, target, kind, 1, alpha_range, rays_per_pair, max_reflections,
                                       ir_seconds))
    return rooms


def mlp_init(seed: int, widths, bias_std: float = 0.0) -> np.ndarray:
    """Flat FP32 parameter vector (W_l [w_l, w_{l-1}] row-major, then b_l,
    layer after layer): He-normal weights (std sqrt(2 / fan_in)) quantised to
    k 2^-e with |k| < 256, so every value is exactly representable in BF16;
    biases N(0, bias_std^2) quantised the same way (0 by default)."""
    rng = np.random.default_rng(seed)

    def quant(x, std):
        if std == 0:
            return np.zeros_like(x)
        e = math.floor(math.log2(std)) - 5               # step = std / 32 .. std / 64
        k = np.clip(np.round(x / 2.0 ** e), -255, 255)
        return (k * 2.0 ** e).astype(np.float32)

    parts = []
    for i, j in zip(widths[:-1], widths[1:]):
        std = math.sqrt(2.0 / i)
        parts.append(quant(rng.standard_normal(i * j) * std, std))
        parts.append(quant(rng.standard_normal(j) * bias_std, bias_std))
    return np.concatenate(parts).astype(np.float32)


def mlp_inputs(seed: int, batch: int, width: int, scale: float = 1.0) -> np.ndarray:
    """[batch, width] FP32 inputs k/64 * scale, |k| <= 192 (exactly BF16 for a
    power-of-two scale)."""
    rng = np.random.default_rng(seed)
    return (rng.integers(-192, 193, size=(batch, width)) / 64.0 * scale).astype(np.float32)


# ----------------------------------------------------------------------------
# air absorption and band filters (inputs to impulse-response assembly)
# ----------------------------------------------------------------------------

def iso9613_beta(temp_c: float = 20.0, rh: float = 50.0, pa_kpa: float = 101.325) -> np.ndarray:
    """Energy air-absorption coefficient per octave band, 1/m, from the ISO
    9613-1 pure-tone attenuation formula at the exact band centres."""
    T = temp_c + 273.15
    T0 = 293.15
    T01 = 273.16
    pr = 101.325
    pa = pa_kpa / pr
    psat = 10.0 ** (-6.8346 * (T01 / T) ** 1.261 + 4.6151)
    h = rh * psat / pa
    frO = pa * (24.0 + 4.04e4 * h * (0.02 + h) / (0.391 + h))
    frN = pa * (T / T0) ** -0.5 * (9.0 + 280.0 * h * math.exp(-4.170 * ((T / T0) ** (-1.0 / 3.0) - 1.0)))
    out = []
    for f in BAND_CENTRES:
        a_db = 8.686 * f * f * (1.84e-11 / pa * (T / T0) ** 0.5 + (T / T0) ** -2.5 * (
            0.01275 * math.exp(-2239.1 / T) / (frO + f * f / frO)
            + 0.1068 * math.exp(-3352.0 / T) / (frN + f * f / frN)))
        out.append(a_db * math.log(10.0) / 10.0)
    return np.array(out, np.float32)


def octave_fir_taps(K: int = 4095, fs: float = 48000.0) -> np.ndarray:
    """[8, K] linear-phase Hann-windowed sinc band-pass taps, band edges
    f_c/sqrt2 .. f_c*sqrt2 around each octave centre (FP64 design, FP32 out)."""
    assert K % 2 == 1
    n = np.arange(K) - (K - 1) / 2.0
    w = 0.5 - 0.5 * np.cos(2 * math.pi * np.arange(K) / (K - 1))
    out = np.empty((8, K))
    for b, fc in enumerate(BAND_CENTRES):
        f1, f2 = fc / math.sqrt(2), min(fc * math.sqrt(2), 0.49 * fs)
        out[b] = w * (2 * f2 / fs * np.sinc(2 * f2 / fs * n) - 2 * f1 / fs * np.sinc(2 * f1 / fs * n))
    return out.astype(np.float32)


def delta_taps(K: int = 1) -> np.ndarray:
    """[8, K] unit impulse at the centre tap (identity filter)."""
    t = np.zeros((8, K), np.float32)
    t[:, (K - 1) // 2] = 1.0
    return t


# ----------------------------------------------------------------------------
# seeded rays, query states and path tables
# ----------------------------------------------------------------------------

def random_unit_dirs(rng, n: int) -> np.ndarray:
    """Isotropic random directions (normalised Gaussians), FP32."""
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d.astype(np.float32)


def surface_query_states(scene: Scene, n: int, seed: int, toward=None):
    """Seeded one-segment query states that start on the mesh, as rays do after
    a reflection: origin = a random point of a random triangle (FP32), direction
    = random unit vector leaving the face on one side (the side facing the point
    ``toward`` when given, else a random side), last plane = that triangle's
    plane id, travelled length uniform in [0, 50] m.
    Returns (origins, dirs, plane, length).
    """
    rng = np.random.default_rng(seed)
    t = rng.integers(0, scene.n_tri, size=n)
    v = scene.vtx.astype(np.float64)[scene.tri[t]]
    a, b = rng.random(n), rng.random(n)
    flip = a + b > 1
    a[flip], b[flip] = 1 - a[flip], 1 - b[flip]
    p = v[:, 0] + a[:, None] * (v[:, 1] - v[:, 0]) + b[:, None] * (v[:, 2] - v[:, 0])
    d = random_unit_dirs(rng, n).astype(np.float64)
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    side = np.where(rng.random(n) < 0.5, 1.0, -1.0)
    if toward is not None:
        side = np.sign(np.einsum("ij,ij->i", np.asarray(toward, np.float64)[None, :] - p, nrm))
        side[side == 0] = 1.0
    s = np.sign(np.einsum("ij,ij->i", d, nrm)) * side
    # keep directions leaving the face on the chosen side
    d = d * np.where(s < 0, -1.0, 1.0)[:, None]
    length = rng.uniform(0.0, 50.0, size=n)
    return (p.astype(np.float32), d.astype(np.float32), scene.plane_id[t].astype(np.int32),
            length.astype(np.float32))


def tie_query_states(scene: Scene, n: int, seed: int):
    """Seeded one-segment query states aimed at mesh vertices (fans of
    triangles that share them) and at shared-edge midpoints, where several
    triangles are crossed at the same or nearly the same point.  Target: a
    random vertex of a random triangle, or the FP32-rounded midpoint of one of
    its edges (half each); origin: the target moved 0.5-3 m along the
    triangle's unit normal (either side) plus a lateral offset of up to 1 m per
    axis (FP32); direction: target - origin (FP32, not normalised, so the
    target lies at parameter 1); no plane excluded, no travelled length.
    Returns (origins, dirs, plane, length)."""
    rng = np.random.default_rng(seed)
    t = rng.integers(0, scene.n_tri, n)
    k = rng.integers(0, 3, n)
    vv = scene.vtx.astype(np.float64)
    v = vv[scene.tri[t, k]]
    w = vv[scene.tri[t, (k + 1) % 3]]
    mid = rng.random(n) < 0.5
    target = np.where(mid[:, None], (v + w) / 2, v).astype(np.float32).astype(np.float64)
    a = vv[scene.tri[t, 0]]
    nrm = np.cross(vv[scene.tri[t, 1]] - a, vv[scene.tri[t, 2]] - a)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    side = np.where(rng.random(n) < 0.5, -1.0, 1.0)[:, None]
    o = (target + side * nrm * rng.uniform(0.5, 3.0, (n, 1)) + rng.uniform(-1.0, 1.0, (n, 3))).astype(np.float32)
    u = (target - o.astype(np.float64)).astype(np.float32)
    return o, u, np.full(n, -1, np.int32), np.zeros(n, np.float32)


def interior_query_states(scene: Scene, n: int, seed: int, lo=None, hi=None):
    """Seeded query states starting inside the scene's bounding box (no last
    plane), random directions, zero travelled length."""
    rng = np.random.default_rng(seed)
    v = scene.vtx.astype(np.float64)
    lo = v.min(0) if lo is None else np.asarray(lo)
    hi = v.max(0) if hi is None else np.asarray(hi)
    o = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
    d = random_unit_dirs(rng, n)
    return o, d, np.full(n, -1, np.int32), np.zeros(n, np.float32)


def synthetic_paths(scene: Scene, n_rays: int, max_reflections: int, n_rcv: int, seed: int,
                    n_prefixes: int = 0, det_per_ray: float = 1.5):
    """Seeded hit-sequence table and detection list with the structure of a
    trace: hit_seq int32 [n_rays, R+1] (triangle ids, -1 padded after a random
    termination), detections int32 [n_det, 3] (ray, segment k, receiver) with k
    below the ray's segment count.  Many rays share prefixes drawn from a pool
    so that image-source keys repeat (dedup work), like beams from a source."""
    rng = np.random.default_rng(seed)
    R1 = max_reflections + 1
    n_prefixes = n_prefixes or max(4, n_rays // 20)
    pool_len = rng.integers(1, R1 + 1, size=n_prefixes)
    pool = rng.integers(0, scene.n_tri, size=(n_prefixes, R1)).astype(np.int32)
    pick = rng.integers(0, n_prefixes, size=n_rays)
    hs = pool[pick].copy()
    seg = pool_len[pick]
    # a quarter of the rays get their own random tail after a shared prefix
    tail = rng.random(n_rays) < 0.25
    cut = rng.integers(0, R1, size=n_rays)
    rnd = rng.integers(0, scene.n_tri, size=(n_rays, R1)).astype(np.int32)
    cols = np.arange(R1)[None, :]
    m = tail[:, None] & (cols >= cut[:, None])
    hs[m] = rnd[m]
    hs[cols >= seg[:, None]] = -1
    # detections
    n_det = int(n_rays * det_per_ray)
    ray = rng.integers(0, n_rays, size=n_det)
    k = (rng.random(n_det) * seg[ray]).astype(np.int64)
    k = np.minimum(k, seg[ray] - 1)
    r = rng.integers(0, n_rcv, size=n_det)
    det = np.stack([ray, k, r], axis=1).astype(np.int32)
    det = np.unique(det, axis=0)
    det = det[rng.permutation(len(det))]
    return hs, det
