"""Seeded scene and deposit-stream generators.

Every generator is deterministic in its seed.  The workloads stand in for
the paper's missing third-party scenes (large rooms, small specular or
refractive objects, many lights; Sec. 6 and 7 of the paper).  Nothing
here is copied from any scene file; all geometry is procedural.

Layouts (shared by both consumers, little endian):
  vertices   float32 (nv, 3)
  tris       int32   (nt, 3)   counter-clockwise seen from the side the
                               geometric normal cross(v1-v0, v2-v0) points to
  tri_mat    int32   (nt,)
  materials  MAT_DTYPE (nm,)   type, albedo rgb, ior, alpha, emission rgb
  point_lights LIGHT_DTYPE (nl,) position, power (watts, rgb)
  camera     CAM_DTYPE scalar  eye, look_at, up, vertical fov in degrees
"""
from dataclasses import dataclass, field
import math

import numpy as np

MAT_LAMBERT, MAT_MIRROR, MAT_DIELECTRIC, MAT_GGX = 0, 1, 2, 3

MAT_DTYPE = np.dtype([("type", "<i4"), ("albedo", "<f4", (3,)), ("ior", "<f4"),
                      ("alpha", "<f4"), ("emission", "<f4", (3,))])
LIGHT_DTYPE = np.dtype([("pos", "<f4", (3,)), ("power", "<f4", (3,))])
CAM_DTYPE = np.dtype([("eye", "<f4", (3,)), ("look_at", "<f4", (3,)),
                      ("up", "<f4", (3,)), ("vfov_deg", "<f4")])


@dataclass
class Scene:
    name: str
    vertices: np.ndarray
    tris: np.ndarray
    tri_mat: np.ndarray
    materials: np.ndarray
    point_lights: np.ndarray
    camera: np.ndarray
    width: int = 64
    height: int = 64
    spp: int = 4
    max_path_len: int = 5
    octree_capacity: int = 4096
    merge_radius: float = 0.01
    seed: int = 1
    scene_id: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_tris(self):
        return int(self.tris.shape[0])

    def bbox(self):
        return self.vertices.min(axis=0), self.vertices.max(axis=0)

    def with_settings(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Scene(**d)


# --------------------------------------------------------------------------
# mesh builders
# --------------------------------------------------------------------------
class _Mesh:
    def __init__(self):
        self.v = []
        self.t = []
        self.m = []
        self.nv = 0

    def add(self, verts, tris, mat):
        verts = np.asarray(verts, np.float64)
        tris = np.asarray(tris, np.int64)
        self.v.append(verts)
        self.t.append(tris + self.nv)
        self.m.append(np.broadcast_to(np.asarray(mat, np.int32), (len(tris),)).copy())
        self.nv += len(verts)

    def quad(self, a, b, c, d, mat):
        """Quad a-b-c-d, counter-clockwise seen from the normal side."""
        self.add([a, b, c, d], [[0, 1, 2], [0, 2, 3]], mat)

    def grid_quad(self, origin, eu, ev, nu, nv, mat):
        """Tessellated parallelogram origin + s*eu + t*ev, normal = eu x ev."""
        o, eu, ev = (np.asarray(x, np.float64) for x in (origin, eu, ev))
        us = np.linspace(0.0, 1.0, nu + 1)
        vs = np.linspace(0.0, 1.0, nv + 1)
        verts = [o + u * eu + v * ev for v in vs for u in us]
        tris = []
        for j in range(nv):
            for i in range(nu):
                a = j * (nu + 1) + i
                b, c, d = a + 1, a + nu + 2, a + nu + 1
                tris += [[a, b, c], [a, c, d]]
        self.add(verts, tris, mat)

    _CORNERS = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                         [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], np.float64)
    # outward-facing quads over the corners above
    _FACES = [[0, 3, 2, 1], [4, 5, 6, 7], [0, 1, 5, 4], [3, 7, 6, 2], [0, 4, 7, 3], [1, 2, 6, 5]]

    @classmethod
    def _box_tris(cls, inward):
        tris = []
        for f in cls._FACES:
            if inward:
                f = f[::-1]
            tris += [[f[0], f[1], f[2]], [f[0], f[2], f[3]]]
        return np.asarray(tris, np.int64)

    def box(self, lo, hi, mat, inward=False):
        lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
        self.add(lo + self._CORNERS * (hi - lo), self._box_tris(inward), mat)

    def boxes(self, lo, hi, mats):
        """Many outward-facing boxes at once: lo, hi (n, 3), mats (n,)."""
        lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
        n = len(lo)
        if n == 0:
            return
        verts = (lo[:, None, :] + self._CORNERS[None] * (hi - lo)[:, None, :]).reshape(-1, 3)
        tris = (self._box_tris(False)[None] + 8 * np.arange(n)[:, None, None]).reshape(-1, 3)
        self.add(verts, tris, np.repeat(np.asarray(mats, np.int32), 12))

    def icosphere(self, center, radius, subdiv, mat):
        v, t = icosphere(subdiv)
        self.add(np.asarray(center) + radius * v, t, mat)

    def build(self):
        v = np.concatenate(self.v).astype(np.float32)
        t = np.concatenate(self.t).astype(np.int32)
        m = np.concatenate(self.m).astype(np.int32)
        return v, t, m


def icosphere(subdiv):
    """Unit icosphere, outward counter-clockwise winding, 20*4^subdiv tris."""
    g = (1.0 + 5 ** 0.5) / 2.0
    v = [[-1, g, 0], [1, g, 0], [-1, -g, 0], [1, -g, 0],
         [0, -1, g], [0, 1, g], [0, -1, -g], [0, 1, -g],
         [g, 0, -1], [g, 0, 1], [-g, 0, -1], [-g, 0, 1]]
    t = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    v = [np.asarray(x, np.float64) / np.linalg.norm(x) for x in v]
    for _ in range(subdiv):
        cache = {}
        nt = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]
        for a, b, c in t:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nt += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        t = nt
    v = np.asarray(v)
    t = np.asarray(t, np.int64)
    # make winding outward
    n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    flip = (n * v[t].mean(axis=1)).sum(axis=1) < 0
    t[flip] = t[flip][:, ::-1]
    return v, t


def torus(center, R, r, nu, nv):
    cu = np.linspace(0, 2 * np.pi, nu, endpoint=False)
    cv = np.linspace(0, 2 * np.pi, nv, endpoint=False)
    verts = []
    for a in cu:
        for b in cv:
            verts.append([(R + r * np.cos(b)) * np.cos(a), r * np.sin(b),
                          (R + r * np.cos(b)) * np.sin(a)])
    verts = np.asarray(verts) + np.asarray(center)
    tris = []
    for i in range(nu):
        for j in range(nv):
            a = i * nv + j
            b = ((i + 1) % nu) * nv + j
            c = ((i + 1) % nu) * nv + (j + 1) % nv
            d = i * nv + (j + 1) % nv
            tris += [[a, d, c], [a, c, b]]
    tris = np.asarray(tris, np.int64)
    # outward orientation test against the tube centre line
    p = verts[tris].mean(axis=1) - np.asarray(center)
    ring = p.copy()
    ring[:, 1] = 0
    ring = ring / np.linalg.norm(ring, axis=1, keepdims=True) * R
    outward = p - ring
    n = np.cross(verts[tris[:, 1]] - verts[tris[:, 0]], verts[tris[:, 2]] - verts[tris[:, 0]])
    flip = (n * outward).sum(axis=1) < 0
    tris[flip] = tris[flip][:, ::-1]
    return verts, tris


def _materials(rows):
    m = np.zeros(len(rows), MAT_DTYPE)
    for i, r in enumerate(rows):
        m[i]["type"] = r.get("type", MAT_LAMBERT)
        m[i]["albedo"] = r.get("albedo", (0.0, 0.0, 0.0))
        m[i]["ior"] = r.get("ior", 1.5)
        m[i]["alpha"] = r.get("alpha", 0.05)
        m[i]["emission"] = r.get("emission", (0.0, 0.0, 0.0))
    return m


def _camera(eye, look_at, up=(0, 1, 0), vfov=60.0):
    c = np.zeros((), CAM_DTYPE)
    c["eye"], c["look_at"], c["up"], c["vfov_deg"] = eye, look_at, up, vfov
    return c


def _no_lights():
    return np.zeros(0, LIGHT_DTYPE)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def tiny_box(width=64, height=64, spp=4, max_path_len=5, seed=1):
    """Closed unit box (12 inward triangles, albedo 0.7, x=0 wall reddish),
    a 0.1 x 0.1 ceiling quad emitting radiance 50, and a mirror icosphere
    r=0.1 (subdivision 2, 320 triangles) at the centre; 64x64, 4 spp,
    path length 5, octree capacity 4096, merge radius 0.01."""
    mats = _materials([
        {"albedo": (0.7, 0.7, 0.7)},                       # 0 white walls
        {"albedo": (0.7, 0.2, 0.2)},                       # 1 red wall
        {"albedo": (0.0, 0.0, 0.0), "emission": (50.0, 50.0, 50.0)},  # 2 light
        {"type": MAT_MIRROR, "albedo": (0.95, 0.95, 0.95)},  # 3 mirror
    ])
    M = _Mesh()
    # inward box faces: floor, ceiling, walls
    M.quad([0, 0, 0], [0, 0, 1], [1, 0, 1], [1, 0, 0], 0)      # floor  y=0, n=+y
    M.quad([0, 1, 0], [1, 1, 0], [1, 1, 1], [0, 1, 1], 0)      # ceil   y=1, n=-y
    M.quad([0, 0, 0], [0, 1, 0], [0, 1, 1], [0, 0, 1], 1)      # x=0,  n=+x (red)
    M.quad([1, 0, 0], [1, 0, 1], [1, 1, 1], [1, 1, 0], 0)      # x=1,  n=-x
    M.quad([0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], 0)      # z=0,  n=+z
    M.quad([0, 0, 1], [0, 1, 1], [1, 1, 1], [1, 0, 1], 0)      # z=1,  n=-z
    y = 0.999
    M.quad([0.45, y, 0.45], [0.55, y, 0.45], [0.55, y, 0.55], [0.45, y, 0.55], 2)  # n=-y
    M.icosphere([0.5, 0.5, 0.5], 0.1, 2, 3)
    v, t, m = M.build()
    return Scene("tiny_box", v, t, m, mats, _no_lights(),
                 _camera([0.5, 0.5, 0.98], [0.5, 0.5, 0.0], (0, 1, 0), 60.0),
                 width=width, height=height, spp=spp, max_path_len=max_path_len,
                 octree_capacity=4096, merge_radius=0.01, seed=seed, scene_id=0)


def room(width=512, height=512, spp=16, max_path_len=8, seed=7, glass_subdiv=5,
         light_subdiv=2):
    """10 x 10 x 3 m room tessellated to ~2k triangles with per-triangle
    grey albedo ~ U[0.3, 0.8], a 1 x 1 m table top at 0.75 m, a glass
    icosphere r=0.15 (IOR 1.5, subdivision 5 = 20480 triangles) resting on
    it and four emissive spheres r=0.02 of radiance 1e3 at 2.6 m above the
    table corners; 512x512, 16 spp, path length 8, octree 2^20 nodes,
    merge radius 0.02."""
    rng = np.random.default_rng(seed)
    M = _Mesh()
    n_wall_mats = 0
    wall_tris = []
    # room shell, inward normals; 18x18 floor and ceiling, 18x5 walls
    shell = _Mesh()
    shell.grid_quad([0, 0, 0], [0, 0, 10], [10, 0, 0], 18, 18, 0)        # floor n=+y
    shell.grid_quad([0, 3, 0], [10, 0, 0], [0, 0, 10], 18, 18, 0)        # ceiling n=-y
    shell.grid_quad([0, 0, 0], [0, 3, 0], [0, 0, 10], 5, 18, 0)          # x=0 n=+x
    shell.grid_quad([10, 0, 0], [0, 0, 10], [0, 3, 0], 18, 5, 0)         # x=10 n=-x
    shell.grid_quad([0, 0, 0], [10, 0, 0], [0, 3, 0], 18, 5, 0)          # z=0 n=+z
    shell.grid_quad([0, 0, 10], [0, 3, 0], [10, 0, 0], 5, 18, 0)         # z=10 n=-z
    sv, st, _ = shell.build()
    n_shell = len(st)
    albedos = rng.uniform(0.3, 0.8, n_shell)
    rows = [{"albedo": (a, a, a)} for a in albedos]
    M.add(sv, st, 0)
    M.m[-1] = np.arange(n_shell, dtype=np.int32)
    base = n_shell
    rows.append({"albedo": (0.55, 0.45, 0.35)})                          # table
    table = base
    rows.append({"type": MAT_DIELECTRIC, "albedo": (1.0, 1.0, 1.0), "ior": 1.5})
    glass = base + 1
    rows.append({"albedo": (0.0, 0.0, 0.0), "emission": (1e3, 1e3, 1e3)})
    lamp = base + 2
    mats = _materials(rows)
    M.box([4.5, 0.70, 4.5], [5.5, 0.75, 5.5], table)
    for cx in (4.55, 5.40):
        for cz in (4.55, 5.40):
            M.box([cx, 0.0, cz], [cx + 0.05, 0.70, cz + 0.05], table)
    M.icosphere([5.0, 0.75 + 0.15, 5.0], 0.15, glass_subdiv, glass)
    for cx in (4.5, 5.5):
        for cz in (4.5, 5.5):
            M.icosphere([cx, 2.6, cz], 0.02, light_subdiv, lamp)
    v, t, m = M.build()
    del n_wall_mats, wall_tris
    return Scene("room", v, t, m, mats, _no_lights(),
                 _camera([5.0, 1.6, 8.0], [5.0, 0.9, 5.0], (0, 1, 0), 50.0),
                 width=width, height=height, spp=spp, max_path_len=max_path_len,
                 octree_capacity=1 << 20, merge_radius=0.02, seed=seed, scene_id=0)


def city_block(width=1024, height=1024, spp=32, max_path_len=10, seed=3, lots=288, lot=2.1, n_lights=1024,
               torus_quads=(200, 125), merge_radius=0.2, octree_capacity=1 << 24, light_height=(150.0, 250.0)):
    """A city block of `lots` x `lots` building lots of `lot` metres (by
    default 288 x 288 lots of 2.1 m: a 605 m square).  Each lot holds one
    extruded box (12 triangles; footprint sides U[0.3, 2.0] m, height
    log-uniform in [0.3, 30] m) placed at random inside the lot at least
    5 cm from its edges, so no two boxes touch or interpenetrate; 5 % of the
    boxes are white GGX alpha 0.05, the rest grey Lambert U[0.3, 0.8].  A
    mirror torus (200 x 125 quads: 50 000 triangles) floats in one corner,
    whose lots stay empty.  Point lights (power U[1, 100] W) hang 150-250 m
    above the ground (aerial lighting: far above every box, a random light
    is seen about 30 degrees up), uniform over the block.
    1024 x 1024, 32 spp, path length 10, octree 2^24 nodes, merge radius
    0.2 m; about 1.05 M triangles."""
    rng = np.random.default_rng(seed)
    B = lots * lot
    rows = [{"albedo": (0.5, 0.5, 0.5)},
            {"type": MAT_MIRROR, "albedo": (0.95, 0.95, 0.95)}]
    n_grey = 16
    for a in np.linspace(0.3, 0.8, n_grey):
        rows.append({"albedo": (a, a, a)})
    rows.append({"type": MAT_GGX, "albedo": (1.0, 1.0, 1.0), "alpha": 0.05})
    ggx = len(rows) - 1
    mats = _materials(rows)
    M = _Mesh()
    M.grid_quad([0, 0, 0], [0, 0, B], [B, 0, 0], 4, 4, 0)
    # one box per lot
    R = min(5.0, 0.1 * B)
    tc = np.array([B - 1.8 * R, 0.6 * R, B - 1.8 * R])
    ix, iz = np.meshgrid(np.arange(lots), np.arange(lots), indexing="ij")
    ix, iz = ix.ravel(), iz.ravel()
    keep = ~((ix + 1) * lot > B - 3.6 * R) | ~((iz + 1) * lot > B - 3.6 * R)
    ix, iz = ix[keep], iz[keep]
    nb = len(ix)
    margin = 0.05
    fmax = min(2.0, lot - 2 * margin)
    fx = rng.uniform(min(0.3, fmax), fmax, nb)
    fz = rng.uniform(min(0.3, fmax), fmax, nb)
    h = np.exp(rng.uniform(np.log(0.3), np.log(30.0), nb))
    x0 = ix * lot + margin + rng.uniform(0, 1, nb) * (lot - 2 * margin - fx)
    z0 = iz * lot + margin + rng.uniform(0, 1, nb) * (lot - 2 * margin - fz)
    lo = np.stack([x0, np.zeros(nb), z0], 1)
    hi = np.stack([x0 + fx, h, z0 + fz], 1)
    corners = np.zeros((nb, 8, 3))
    for i, (sx, sy, sz) in enumerate([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                                      (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]):
        corners[:, i, 0] = np.where(sx, hi[:, 0], lo[:, 0])
        corners[:, i, 1] = np.where(sy, hi[:, 1], lo[:, 1])
        corners[:, i, 2] = np.where(sz, hi[:, 2], lo[:, 2])
    faces = [[0, 3, 2, 1], [4, 5, 6, 7], [0, 1, 5, 4], [3, 7, 6, 2], [0, 4, 7, 3], [1, 2, 6, 5]]
    ft = []
    for f in faces:
        ft += [[f[0], f[1], f[2]], [f[0], f[2], f[3]]]
    ft = np.asarray(ft)
    bmat = np.where(rng.uniform(size=nb) < 0.05, ggx,
                    2 + rng.integers(0, n_grey, nb)).astype(np.int32)
    bv = corners.reshape(-1, 3)
    btris = (np.arange(nb)[:, None, None] * 8 + ft[None]).reshape(-1, 3)
    M.v.append(bv)
    base = sum(len(a) for a in M.v[:-1])
    M.t.append(btris + base)
    M.m.append(np.repeat(bmat, 12))
    tv, tt = torus(tc, R, 0.3 * R, torus_quads[0], torus_quads[1])
    M.add(tv, tt, 1)
    v, t, m = M.build()
    lights = np.zeros(n_lights, LIGHT_DTYPE)
    lights["pos"][:, 0] = rng.uniform(0, B, n_lights)
    lights["pos"][:, 1] = rng.uniform(light_height[0], light_height[1], n_lights)
    lights["pos"][:, 2] = rng.uniform(0, B, n_lights)
    p = rng.uniform(1.0, 100.0, n_lights)
    lights["power"] = np.stack([p, p, p], 1)
    return Scene("city_block", v, t, m, mats, lights,
                 _camera([-0.05 * B, 0.45 * B, -0.05 * B], [0.5 * B, 0.0, 0.5 * B], (0, 1, 0), 45.0),
                 width=width, height=height, spp=spp, max_path_len=max_path_len,
                 octree_capacity=octree_capacity, merge_radius=merge_radius, seed=seed, scene_id=0)


def city_lots(width=48, height=48, spp=4, lots=12, n_lights=64, seed=3):
    """The city block's recipe on a small block (12 x 12 lots of 2.1 m, 64
    point lights, a 24 x 12-quad mirror torus): GGX boxes, a mirror and
    power-sampled point lights at path length 10, small enough for the
    brute-force oracle."""
    return city_block(width=width, height=height, spp=spp, seed=seed, lots=lots, n_lights=n_lights,
                      torus_quads=(24, 12), octree_capacity=1 << 20)


def _box_room_scene(rng, n_target, n_lights, res, spp, seed, scene_id):
    rows = [{"albedo": (0.6, 0.6, 0.6)}, {"albedo": (0.7, 0.3, 0.3)},
            {"albedo": (0.0, 0.0, 0.0), "emission": (200.0, 200.0, 200.0)},
            {"type": MAT_MIRROR, "albedo": (0.9, 0.9, 0.9)},
            {"type": MAT_DIELECTRIC, "albedo": (1.0, 1.0, 1.0), "ior": 1.5}]
    mats = _materials(rows)
    M = _Mesh()
    L = 4.0
    M.box([0, 0, 0], [L, 2.5, L], 0, inward=True)
    # interior random boxes up to the triangle budget
    n_boxes = max(0, (n_target - 12 - n_lights * 80) // 12)
    lo = np.empty((int(n_boxes), 3))
    hi = np.empty((int(n_boxes), 3))
    bm = np.empty(int(n_boxes), np.int32)
    for i in range(int(n_boxes)):
        s = rng.uniform(0.02, 0.3, 3)
        c = rng.uniform([0.2, 0.0, 0.2], [L - 0.2, 1.5, L - 0.2])
        lo[i], hi[i] = c, c + s
        bm[i] = int(rng.integers(0, 5)) if rng.uniform() < 0.1 else int(rng.integers(0, 2))
    M.boxes(lo, hi, bm)
    for _ in range(int(n_lights)):
        c = rng.uniform([0.3, 1.9, 0.3], [L - 0.3, 2.3, L - 0.3])
        M.icosphere(c, 0.02, 1, 2)
    v, t, m = M.build()
    return Scene(f"batch_room_{scene_id}", v, t, m, mats, _no_lights(),
                 _camera([L / 2, 1.3, L - 0.1], [L / 2, 0.8, 0.0], (0, 1, 0), 60.0),
                 width=res, height=res, spp=spp, max_path_len=8,
                 octree_capacity=1 << 18, merge_radius=0.002 * float(np.linalg.norm([L, 2.5, L])),
                 seed=seed, scene_id=scene_id)


def batch_rooms(n_scenes=64, seed=4):
    """64 box rooms: triangle count log-uniform on [1e3, 5e5] (interior
    random boxes), 1-256 sphere lights, square resolution U[64, 512],
    spp U{4..32}, path length 8, scene s has scene id s."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scenes):
        n_target = int(np.exp(rng.uniform(np.log(1e3), np.log(5e5))))
        n_lights = int(rng.integers(1, 257))
        n_lights = min(n_lights, max(1, (n_target - 12) // 80))
        res = int(rng.integers(64, 513))
        spp = int(rng.integers(4, 33))
        out.append(_box_room_scene(rng, n_target, n_lights, res, spp, seed, s))
    return out


def box_room(n_tris=3000, n_lights=4, res=96, spp=4, seed=4, scene_id=0):
    """One box room of the batch recipe with chosen sizes (the interior
    boxes and light positions are drawn from `seed` and `scene_id`)."""
    rng = np.random.default_rng([seed, scene_id])
    return _box_room_scene(rng, n_tris, n_lights, res, spp, seed, scene_id)


def furnace_sphere(radius=1.0, albedo=0.5, emission=1.0, subdiv=4, width=16, height=16,
                   max_path_len=5, spp=4, seed=11):
    """Closed sphere with inward normals; its interior is Lambertian with
    albedo `albedo` and emits radiance `emission`; the camera sits at the
    centre.  A tessellated sphere is a closed convex polyhedron; the
    closed forms used by the tests hold for any closed convex emitter
    that is its own Lambertian surface, see tests."""
    v, t = icosphere(subdiv)
    t = t[:, ::-1].copy()                    # inward
    mats = _materials([{"albedo": (albedo,) * 3, "emission": (emission,) * 3}])
    return Scene("furnace", (v * radius).astype(np.float32), t.astype(np.int32),
                 np.zeros(len(t), np.int32), mats, _no_lights(),
                 _camera([0.0, 0.0, 0.0], [0.0, 0.0, -1.0], (0, 1, 0), 60.0),
                 width=width, height=height, spp=spp, max_path_len=max_path_len,
                 octree_capacity=1 << 16, merge_radius=0.05 * radius, seed=seed, scene_id=0)


def disk_light_plane(disk_radius=0.5, height=1.0, radiance=2.0, albedo=0.6, n_seg=64,
                     width=16, height_px=16, spp=16, seed=12, plane_half=4.0):
    """A one-sided regular n_seg-gon emitter of circumradius `disk_radius`
    facing down at `height` above a grey Lambertian plane; the camera
    sits halfway between them on the axis and looks straight down with
    a narrow field of view.  Path length 2 (direct light only)."""
    mats = _materials([{"albedo": (albedo,) * 3},
                       {"albedo": (0.0,) * 3, "emission": (radiance,) * 3}])
    M = _Mesh()
    M.quad([-plane_half, 0, -plane_half], [-plane_half, 0, plane_half],
           [plane_half, 0, plane_half], [plane_half, 0, -plane_half], 0)   # n=+y
    ang = np.linspace(0, 2 * np.pi, n_seg, endpoint=False)
    ring = np.stack([disk_radius * np.cos(ang), np.full(n_seg, height),
                     disk_radius * np.sin(ang)], 1)
    verts = np.concatenate([[[0.0, height, 0.0]], ring])
    tris = [[0, 1 + i, 1 + (i + 1) % n_seg] for i in range(n_seg)]
    M.add(verts, tris, 1)
    v, t, m = M.build()
    # orient emitter triangles to face -y
    n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    flip = (m == 1) & (n[:, 1] > 0)
    t[flip] = t[flip][:, ::-1]
    return Scene("disk_light", v, t, m, mats, _no_lights(),
                 _camera([0.0, height * 0.5, 0.0], [0.0, 0.0, 0.0], (0, 0, 1), 20.0),
                 width=width, height=height_px, spp=spp, max_path_len=2,
                 octree_capacity=1 << 14, merge_radius=0.01, seed=seed, scene_id=0)


def point_light_plane(height=1.0, power=40.0, albedo=0.6, width=8, height_px=8, spp=16, seed=13,
                      plane_half=4.0, merge_radius=0.05):
    """An isotropic point light of `power` watts at `height` above a grey
    Lambertian plane; the camera sits halfway between them on the axis and
    looks straight down with a narrow field of view.  Path length 2
    (direct light only).  A small black triangle above a far corner gives
    the scene a non-flat bounding box; it shades nothing the camera sees."""
    mats = _materials([{"albedo": (albedo,) * 3}, {"albedo": (0.0,) * 3}])
    M = _Mesh()
    M.quad([-plane_half, 0, -plane_half], [-plane_half, 0, plane_half],
           [plane_half, 0, plane_half], [plane_half, 0, -plane_half], 0)   # n=+y
    c = plane_half * 0.9
    M.add([[c, 2 * height, c], [c - 0.1, 2 * height, c], [c, 2 * height, c - 0.1]], [[0, 1, 2]], 1)
    v, t, m = M.build()
    lights = np.zeros(1, LIGHT_DTYPE)
    lights["pos"][0] = (0.0, height, 0.0)
    lights["power"][0] = (power,) * 3
    return Scene("point_light", v, t, m, mats, lights,
                 _camera([0.0, height * 0.5, 0.0], [0.0, 0.0, 0.0], (0, 0, 1), 20.0),
                 width=width, height=height_px, spp=spp, max_path_len=2,
                 octree_capacity=1 << 14, merge_radius=merge_radius, seed=seed, scene_id=0)


def random_triangle_soup(n_tris, seed, extent=1.0):
    """Random triangles in [0, extent]^3 (for intersection tests)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 0.9, (n_tris, 1, 3)) * extent
    d = rng.normal(0.0, 0.15 * extent, (n_tris, 3, 3))
    v = (c + d).reshape(-1, 3).astype(np.float32)
    t = np.arange(3 * n_tris, dtype=np.int32).reshape(-1, 3)
    return v, t


def deposit_stream(n, seed, kind="mixed"):
    """float32 (n,3) positions in [0,1]^3 for octree tests: points on a few
    planes (axis-aligned and tilted) plus a clustered blob."""
    rng = np.random.default_rng(seed)
    pts = []
    k = n // 4
    a = rng.uniform(0.05, 0.95, (k, 2))
    pts.append(np.stack([a[:, 0], np.full(k, 0.3), a[:, 1]], 1))           # y=0.3 plane
    a = rng.uniform(0.05, 0.95, (k, 2))
    pts.append(np.stack([np.full(k, 0.71), a[:, 0], a[:, 1]], 1))          # x=0.71 plane
    a = rng.uniform(0.1, 0.9, (k, 2))
    z = 0.2 + 0.5 * a[:, 0] + 0.1 * a[:, 1]
    pts.append(np.stack([a[:, 0], a[:, 1], z], 1))                          # tilted plane
    r = n - 3 * k
    pts.append(np.clip(rng.normal(0.5, 0.04, (r, 3)), 0.01, 0.99))         # blob
    p = np.concatenate(pts)
    p = p[rng.permutation(len(p))]
    return p.astype(np.float32)


def plane_deposits(n, seed, normal=(0.0, 1.0, 0.0), offset=0.437, lo=0.0, hi=1.0):
    """n float32 points uniform on the plane {x : <normal, x> = offset}
    restricted to the square [lo, hi] in the two coordinates other than
    the normal's largest component."""
    rng = np.random.default_rng(seed)
    nrm = np.asarray(normal, np.float64)
    nrm = nrm / np.linalg.norm(nrm)
    ax = int(np.argmax(np.abs(nrm)))
    o = [i for i in range(3) if i != ax]
    uv = rng.uniform(lo, hi, (n, 2))
    p = np.zeros((n, 3))
    p[:, o[0]] = uv[:, 0]
    p[:, o[1]] = uv[:, 1]
    p[:, ax] = (offset - nrm[o[0]] * uv[:, 0] - nrm[o[1]] * uv[:, 1]) / nrm[ax]
    return p.astype(np.float32)


def sphere_deposits(n, seed, center=(0.5, 0.5, 0.5), radius=0.1):
    """n float32 points uniform on the sphere |x - center| = radius, and
    their float32 outward unit normals."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    p = np.asarray(center, np.float64) + radius * v
    return p.astype(np.float32), v.astype(np.float32)


def query_points(n, seed, lo=0.0, hi=1.0):
    """Random float32 query positions and unit float32 normals."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(lo, hi, (n, 3)).astype(np.float32)
    nrm = rng.normal(size=(n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return p, nrm.astype(np.float32)


def scene_by_name(name, **kw):
    return {"tiny_box": tiny_box, "room": room, "city_block": city_block,
            "furnace": furnace_sphere, "disk_light": disk_light_plane, "city_lots": city_lots}[name](**kw)
