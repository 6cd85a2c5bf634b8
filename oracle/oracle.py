"""ctypes wrapper of the FP64 C oracle (``neb_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``.  The product library never imports
this module and shares no code with it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "neb_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libneb_oracle.so")
_lib = None


def build(force=False):
    """Compile the oracle with gcc (OpenMP, no FP contraction)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class Material(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("albedo", ctypes.c_float * 3), ("ior", ctypes.c_float),
                ("alpha", ctypes.c_float), ("emission", ctypes.c_float * 3)]


class Params(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("max_path_len", ctypes.c_int32), ("octree_capacity", ctypes.c_int32),
                ("merge_radius", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("scene_id", ctypes.c_uint32), ("density_mode", ctypes.c_int32),
                ("analytic_rho0", ctypes.c_double), ("analytic_cam_weight", ctypes.c_double),
                ("enable_photons", ctypes.c_int32),
                ("win_x0", ctypes.c_int32), ("win_y0", ctypes.c_int32),
                ("win_x1", ctypes.c_int32), ("win_y1", ctypes.c_int32),
                ("n_threads", ctypes.c_int32), ("record_paths", ctypes.c_int32),
                ("light_photons", ctypes.c_int32), ("density_radius", ctypes.c_double),
                ("knn_k", ctypes.c_int32), ("nee_radius", ctypes.c_double),
                ("freeze_after", ctypes.c_int32), ("density_hook", ctypes.c_void_p)]


# void hook(n, pos (n*3), nrm (n*3), pixel (n), depth (n), iteration, rho (n, in/out))
DENSITY_HOOK = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(ctypes.c_double))


class Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("paths", "vertices", "photons", "photon_segments", "merges", "nee_visible",
                 "events", "rays")] + \
               [(k, ctypes.c_int64) for k in
                ("oct_nodes", "oct_depth", "oct_overflow", "oct_ledger", "oct_deposits",
                 "oct_capacity", "oct_rejected")] + \
               [("light_photons", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


RECORD_DTYPE = np.dtype([("type", "<i4"), ("mat", "<i4"), ("prim", "<i4"), ("pos", "<f4", (3,))])

DENSITY_SINGLE, DENSITY_ROBUST, DENSITY_ANALYTIC, DENSITY_RADIUS, DENSITY_KNN = 0, 1, 3, 4, 5

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_philox4x32_10.argtypes = [_P, _P, _P]
        L.orc_exact_area.argtypes = [_P, _P, _P, _P]
        L.orc_exact_area.restype = ctypes.c_double
        L.orc_octree_create.argtypes = [_P, _P, ctypes.c_int32]
        L.orc_octree_create.restype = _P
        L.orc_octree_destroy.argtypes = [_P]
        L.orc_octree_box.argtypes = [_P, _P, _P]
        L.orc_octree_set_iteration.argtypes = [_P, ctypes.c_int32]
        L.orc_octree_clear_counters.argtypes = [_P]
        L.orc_octree_increment.argtypes = [_P, _P, ctypes.c_int64]
        L.orc_octree_density.argtypes = [_P, _P, _P, ctypes.c_int32]
        L.orc_octree_density.restype = ctypes.c_double
        L.orc_octree_density_batch.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, _P]
        L.orc_octree_export.argtypes = [_P, _P, ctypes.c_int32, _P]
        L.orc_octree_export.restype = ctypes.c_int32
        L.orc_scene_create.argtypes = [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, ctypes.c_int32,
                                       _P, ctypes.c_int32, _P]
        L.orc_scene_create.restype = _P
        L.orc_scene_destroy.argtypes = [_P]
        L.orc_scene_bounds.argtypes = [_P, _P, _P]
        L.orc_closest_hit.argtypes = [_P, _P, _P, _P]
        L.orc_closest_hit.restype = ctypes.c_int32
        L.orc_render.argtypes = [_P, ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32, _P,
                                 _P, _P, _P, _P, ctypes.POINTER(Stats), _P]
        L.orc_render.restype = ctypes.c_int32
        L.orc_bsdf_eval.argtypes = [ctypes.POINTER(Material), _P, _P, _P, _P, _P]
        L.orc_bsdf_sample.argtypes = [ctypes.POINTER(Material), _P, _P, _P, _P, _P, _P]
        L.orc_bsdf_sample.restype = ctypes.c_int32
        L.orc_path_technique_densities.argtypes = [ctypes.c_int32, _P, _P, _P, ctypes.c_double,
                                                   ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_int32, ctypes.c_double, _P]
        L.orc_path_technique_densities.restype = ctypes.c_int32
        L.orc_point_density.argtypes = [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_int32, _P]
        L.orc_point_density.restype = ctypes.c_int32
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


# ---------------------------------------------------------------------------
def philox(counter, key):
    c = np.ascontiguousarray(counter, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def exact_area(bmin, bmax, p, n):
    a = [np.ascontiguousarray(x, np.float64) for x in (bmin, bmax, p, n)]
    return lib().orc_exact_area(*[_ptr(x) for x in a])


def material(type=0, albedo=(0.5, 0.5, 0.5), ior=1.5, alpha=0.05, emission=(0, 0, 0)):
    m = Material()
    m.type = type
    m.albedo[:] = albedo
    m.ior = ior
    m.alpha = alpha
    m.emission[:] = emission
    return m


def bsdf_eval(mat, n, wi, wo):
    a = [np.ascontiguousarray(x, np.float64) for x in (n, wi, wo)]
    f = np.zeros(3)
    pdf = np.zeros(1)
    lib().orc_bsdf_eval(ctypes.byref(mat), *[_ptr(x) for x in a], _ptr(f), _ptr(pdf))
    return f, float(pdf[0])


def bsdf_sample(mat, n, wi, u):
    a = [np.ascontiguousarray(x, np.float64) for x in (n, wi, u)]
    d = np.zeros(3)
    w = np.zeros(3)
    pdf = np.zeros(1)
    ev = lib().orc_bsdf_sample(ctypes.byref(mat), *[_ptr(x) for x in a], _ptr(d), _ptr(w), _ptr(pdf))
    return ev, d, w, float(pdf[0])


def technique_densities(pos, nrm, mats, p_light, hittable, rho, radius, photons=True, n_lp=None):
    """Densities of every technique that can form the explicit path `pos`
    (camera first, light last): [e, E, P_1 .. P_{L-2}], followed by
    [LP_1 .. LP_{L-1}] when `n_lp` (light photons per iteration) is given."""
    L = len(pos) - 1
    pos = np.ascontiguousarray(pos, np.float64)
    nrm = np.ascontiguousarray(nrm, np.float64)
    arr = (Material * max(1, L - 1))(*mats) if L > 1 else (Material * 1)()
    out = np.zeros(2 * L + 2)
    n = lib().orc_path_technique_densities(L, _ptr(pos), _ptr(nrm), arr, p_light, int(hittable),
                                           rho, radius, int(photons), float(n_lp or 0.0), _ptr(out))
    if n_lp is None:
        n = 2 + max(0, L - 2)
    return out[:n]


def point_density(points, queries, mode, radius, k=4):
    """Fixed-radius (mode 4) or k-nearest-neighbour (mode 5) density at the
    query points over the point set (per unit area)."""
    pts = np.ascontiguousarray(points, np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(queries, np.float64).reshape(-1, 3)
    out = np.zeros(len(q))
    if lib().orc_point_density(_ptr(pts), len(pts), _ptr(q), len(q), int(mode), float(radius), int(k), _ptr(out)):
        raise ValueError("bad point-density arguments")
    return out


class Octree:
    """Sequential density octree (FP32 cell addressing, FP64 areas)."""

    def __init__(self, smin, smax, capacity):
        self._smin = np.ascontiguousarray(smin, np.float32)
        self._smax = np.ascontiguousarray(smax, np.float32)
        self.h = lib().orc_octree_create(_ptr(self._smin), _ptr(self._smax), int(capacity))
        if not self.h:
            raise ValueError("bad octree parameters")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_octree_destroy(self.h)
            self.h = None

    def set_iteration(self, it):
        lib().orc_octree_set_iteration(self.h, int(it))

    def clear_counters(self):
        lib().orc_octree_clear_counters(self.h)

    def increment(self, pos):
        p = np.ascontiguousarray(pos, np.float32).reshape(-1, 3)
        lib().orc_octree_increment(self.h, _ptr(p), p.shape[0])

    def density(self, pos, nrm, robust=True):
        p = np.ascontiguousarray(pos, np.float32).reshape(-1, 3)
        n = np.ascontiguousarray(nrm, np.float32).reshape(-1, 3)
        out = np.zeros(p.shape[0])
        lib().orc_octree_density_batch(self.h, _ptr(p), _ptr(n), p.shape[0], int(robust), _ptr(out))
        return out

    def density_f64(self, p, n, robust=True):
        a = np.ascontiguousarray(p, np.float64)
        b = np.ascontiguousarray(n, np.float64)
        return lib().orc_octree_density(self.h, _ptr(a), _ptr(b), int(robust))

    def box(self):
        """(min_bound, size_inv) float32 of the cell addressing."""
        lo = np.zeros(3, np.float32)
        inv = np.zeros(3, np.float32)
        lib().orc_octree_box(self.h, _ptr(lo), _ptr(inv))
        return lo, inv

    def export(self):
        info = np.zeros(8, np.int64)
        lib().orc_octree_export(self.h, None, 0, _ptr(info))
        nodes = np.zeros(int(info[0]), np.int32)
        lib().orc_octree_export(self.h, _ptr(nodes), nodes.size, _ptr(info))
        keys = ("capacity", "allocated", "depth", "ledger", "deposits", "overflow", "rejected",
                "block_iter_sum")
        return nodes, dict(zip(keys, (int(x) for x in info)))


class OracleScene:
    def __init__(self, scene):
        self.scene = scene
        self._keep = [np.ascontiguousarray(scene.vertices, np.float32),
                      np.ascontiguousarray(scene.tris, np.int32),
                      np.ascontiguousarray(scene.tri_mat, np.int32),
                      np.ascontiguousarray(scene.materials),
                      np.ascontiguousarray(scene.point_lights),
                      np.ascontiguousarray(scene.camera)]
        v, t, m, mats, pl, cam = self._keep
        self.h = lib().orc_scene_create(_ptr(v), v.shape[0], _ptr(t), _ptr(m), t.shape[0],
                                        _ptr(mats), mats.shape[0], _ptr(pl), pl.shape[0], _ptr(cam))
        if not self.h:
            raise ValueError("bad scene")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_scene_destroy(self.h)
            self.h = None

    def bounds(self):
        a = np.zeros(3, np.float32)
        b = np.zeros(3, np.float32)
        lib().orc_scene_bounds(self.h, _ptr(a), _ptr(b))
        return a, b

    def closest_hit(self, o, d):
        o = np.ascontiguousarray(o, np.float64)
        d = np.ascontiguousarray(d, np.float64)
        t = np.zeros(1)
        prim = lib().orc_closest_hit(self.h, _ptr(o), _ptr(d), _ptr(t))
        return prim, float(t[0])


def make_params(scene, density_mode=DENSITY_ROBUST, enable_photons=True, window=None, n_threads=0,
                record=False, rho0=0.0, cam_weight=0.0, light_photons=0, density_radius=0.0, knn_k=8,
                nee_radius=0.0, freeze_after=0, **over):
    p = Params()
    p.width = over.get("width", scene.width)
    p.height = over.get("height", scene.height)
    p.max_path_len = over.get("max_path_len", scene.max_path_len)
    p.octree_capacity = over.get("octree_capacity", scene.octree_capacity)
    p.merge_radius = over.get("merge_radius", scene.merge_radius)
    p.seed = over.get("seed", scene.seed)
    p.scene_id = over.get("scene_id", scene.scene_id)
    p.density_mode = density_mode
    p.analytic_rho0 = rho0
    p.analytic_cam_weight = cam_weight
    p.enable_photons = int(enable_photons)
    if window is not None:
        p.win_x0, p.win_y0, p.win_x1, p.win_y1 = window
    p.n_threads = n_threads
    p.record_paths = int(record)
    p.light_photons = int(light_photons)
    p.density_radius = float(density_radius)
    p.knn_k = int(knn_k)
    p.nee_radius = float(nee_radius)
    p.freeze_after = int(freeze_after)
    p.density_hook = None
    return p


def render(scene, n_iter=None, first_iter=1, density_mode=DENSITY_ROBUST, enable_photons=True,
           window=None, n_threads=0, record=False, rho0=0.0, cam_weight=0.0, oscene=None,
           octree=None, light_photons=0, density_radius=0.0, knn_k=8, nee_radius=0.0, freeze_after=0,
           density_hook=None, **over):
    """Render `n_iter` progressive iterations (1 spp each).  Returns a dict
    with per-technique image sums (H, W, 3): e, E, P and, with
    `light_photons` > 0 conventional photons per iteration, LP; their sum,
    the mean image, the stats and, if requested, the first iteration's path
    records.  freeze_after > 0 stops the octree's deposits after that
    iteration (it keeps that iteration's scalars); density_hook(pos, nrm,
    pixel, depth, iteration, rho) may overwrite each iteration's densities
    (numpy arrays; rho holds the provider's values)."""
    osc = oscene or OracleScene(scene)
    prm = make_params(scene, density_mode, enable_photons, window, n_threads, record, rho0,
                      cam_weight, light_photons, density_radius, knn_k, nee_radius, freeze_after, **over)
    cb = None
    if density_hook is not None:
        def _hook(n, pos, nrm, pixel, depth, it, rho):
            P = np.ctypeslib.as_array(pos, (n, 3))
            N = np.ctypeslib.as_array(nrm, (n, 3))
            px = np.ctypeslib.as_array(pixel, (n,))
            dp = np.ctypeslib.as_array(depth, (n,))
            r = np.ctypeslib.as_array(rho, (n,))
            r[:] = density_hook(P.copy(), N.copy(), px.copy(), dp.copy(), int(it), r.copy())
        cb = DENSITY_HOOK(_hook)
        prm.density_hook = ctypes.cast(cb, ctypes.c_void_p)
    n_iter = scene.spp if n_iter is None else n_iter
    oct_ = octree
    if oct_ is None and density_mode in (DENSITY_SINGLE, DENSITY_ROBUST):
        lo, hi = osc.bounds()
        oct_ = Octree(lo, hi, prm.octree_capacity)
    H, W = prm.height, prm.width
    imgs = {k: np.zeros((H, W, 3)) for k in ("e", "E", "P", "LP")}
    st = Stats()
    rec = None
    if record:
        x0, y0, x1, y1 = window if window is not None else (0, 0, W, H)
        rec = np.zeros(((x1 - x0) * (y1 - y0), prm.max_path_len), RECORD_DTYPE)
    rc = lib().orc_render(osc.h, ctypes.byref(prm), int(n_iter), int(first_iter),
                          oct_.h if oct_ is not None else None,
                          _ptr(imgs["e"]), _ptr(imgs["E"]), _ptr(imgs["P"]), _ptr(imgs["LP"]),
                          ctypes.byref(st),
                          _ptr(rec) if rec is not None else None)
    if rc != 0:
        raise RuntimeError("oracle render failed")
    total = imgs["e"] + imgs["E"] + imgs["P"] + imgs["LP"]
    return {"sum": total, "mean": total / max(1, n_iter), "tech": imgs, "stats": st.as_dict(),
            "records": rec, "octree": oct_, "n_iter": n_iter}
