"""Thin ctypes binding of libneb.so (include/neb.h).

Argument marshalling only: every step of the path runs in the library's
HIP kernels.  torch is used for device buffers and streams.  The binding
refuses to run without the built library (no CPU fallback exists).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libneb.so")
_lib = None

NEB_OK = 0
DENSITY_OCTREE, DENSITY_OCTREE_ROBUST, DENSITY_MLP, DENSITY_ANALYTIC, DENSITY_RADIUS, DENSITY_KNN = 0, 1, 2, 3, 4, 5
MLP_PARAMS = 13569
FLAG_SINGLE_THREAD_OCTREE, FLAG_RECORD_PATHS, FLAG_NO_PHOTONS = 1, 2, 4

# every symbol the header declares
EXPORTS = [
    "neb_create", "neb_create_batch", "neb_set_scene", "neb_set_batch_scene", "neb_render", "neb_use_graph",
    "neb_autotune", "neb_set_launch_config", "neb_get_launch_config", "neb_get_image", "neb_get_scene_image",
    "neb_get_technique_images", "neb_get_scene_technique_images", "neb_get_scene_light_photon_image",
    "neb_query_density", "neb_point_density", "neb_point_density_noalloc", "neb_get_stats", "neb_get_path_records", "neb_get_octree", "neb_get_scene_octree",
    "neb_profile_kernels", "neb_get_kernel_profile", "neb_reset",
    "neb_destroy", "neb_status_string", "neb_last_error",
    "neb_configure_mlp", "neb_get_mlp_status", "neb_get_mlp_weights", "neb_set_mlp_model", "neb_get_mlp_gates", "neb_mlp_create", "neb_mlp_set_normalization",
    "neb_mlp_infer", "neb_mlp_gradient", "neb_mlp_train_step", "neb_mlp_get_params", "neb_mlp_destroy",
    "neb_octree_create", "neb_octree_set_iteration", "neb_octree_increment", "neb_octree_density",
    "neb_octree_clear_counters", "neb_octree_export", "neb_octree_destroy", "neb_atomic_probe", "neb_gather_probe",
]


class NebError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("max_path_len", ctypes.c_int32),
                ("octree_capacity", ctypes.c_int32), ("merge_radius", ctypes.c_float),
                ("seed", ctypes.c_uint32), ("scene_id", ctypes.c_uint32), ("density_mode", ctypes.c_int32),
                ("analytic_rho0", ctypes.c_float), ("analytic_cam_weight", ctypes.c_float),
                ("flags", ctypes.c_int32), ("spp", ctypes.c_int32), ("light_photons", ctypes.c_int32),
                ("density_radius", ctypes.c_float), ("knn_k", ctypes.c_int32), ("nee_radius", ctypes.c_float)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("bvh_stack", ctypes.c_int32), ("trace_blocks_per_cu", ctypes.c_int32),
                ("nee_blocks_per_cu", ctypes.c_int32), ("photon_blocks_per_cu", ctypes.c_int32),
                ("photon_order", ctypes.c_int32), ("concurrent", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "iterations", "paths", "vertices", "photons", "photon_segments", "merges", "nee_visible", "events",
        "rays", "oct_capacity", "oct_allocated", "oct_depth", "oct_overflow", "oct_ledger", "oct_deposits",
        "oct_rejected", "oct_lost", "photon_items", "photon_continued", "grid_cells", "candidates",
        "camera_rays", "shadow_rays", "bvh_nodes", "bvh_tris", "light_photons", "bvh_nodes_camera",
        "bvh_nodes_photon", "bvh_nodes_shadow", "bvh_tris_camera", "bvh_tris_photon", "bvh_tris_shadow")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class MlpParams(ctypes.Structure):
    _fields_ = [("train_iterations", ctypes.c_int32), ("steps_per_iteration", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("probe_every", ctypes.c_int32),
                ("probes", ctypes.c_int32), ("max_rel_error", ctypes.c_float), ("seed", ctypes.c_uint32)]


MLP_DEFAULTS = dict(train_iterations=4, steps_per_iteration=250, batch=65536, lr=2e-3, beta1=0.9, beta2=0.999,
                    eps=1e-8, probe_every=8, probes=4096, max_rel_error=0.1, seed=1)


class MlpStatus(ctypes.Structure):
    _fields_ = [("phase", ctypes.c_int32), ("adam_steps", ctypes.c_int64), ("last_loss", ctypes.c_double),
                ("mu", ctypes.c_float), ("sigma", ctypes.c_float), ("probes", ctypes.c_int64),
                ("probes_bad", ctypes.c_int64), ("regions_probed", ctypes.c_int64),
                ("regions_disabled", ctypes.c_int64), ("fallback_queries", ctypes.c_int64),
                ("probes_served", ctypes.c_int64), ("probes_served_bad", ctypes.c_int64)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t in (ctypes.c_double, ctypes.c_float) else int(getattr(self, k)))
                for k, t in self._fields_}


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


RECORD_DTYPE = np.dtype([("type", "<i4"), ("mat", "<i4"), ("prim", "<i4"), ("pos", "<f4", (3,))])
OCT_INFO_KEYS = ("capacity", "allocated", "depth", "ledger", "deposits", "overflow", "rejected", "lost")

_P = ctypes.c_void_p


def lib():
    """Load libneb.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NebError(f"{LIB_PATH} is missing: build it with paper_1909_00573_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        sig = {
            "neb_create": ([ctypes.POINTER(Params), ctypes.POINTER(_P)], i32),
            "neb_create_batch": ([ctypes.POINTER(Params), i32, ctypes.POINTER(_P)], i32),
            "neb_set_scene": ([_P, _P, i32, _P, _P, i32, _P, i32, _P, i32, _P], i32),
            "neb_set_batch_scene": ([_P, i32, _P, i32, _P, _P, i32, _P, i32, _P, i32, _P], i32),
            "neb_render": ([_P, i32, _P], i32),
            "neb_use_graph": ([_P, i32], i32),
            "neb_autotune": ([_P, i32, _P, ctypes.POINTER(LaunchConfig)], i32),
            "neb_set_launch_config": ([_P, ctypes.POINTER(LaunchConfig)], i32),
            "neb_get_launch_config": ([_P, ctypes.POINTER(LaunchConfig)], i32),
            "neb_get_image": ([_P, _P, i32, _P], i32),
            "neb_get_scene_image": ([_P, i32, _P, i32, _P], i32),
            "neb_get_technique_images": ([_P, _P, _P, _P, i32, _P], i32),
            "neb_get_scene_technique_images": ([_P, i32, _P, _P, _P, i32, _P], i32),
            "neb_get_scene_light_photon_image": ([_P, i32, _P, i32, _P], i32),
            "neb_query_density": ([_P, _P, _P, i32, _P, i32, _P], i32),
            "neb_point_density": ([_P, i32, _P, i32, i32, ctypes.c_float, i32, _P, _P], i32),
            "neb_point_density_noalloc": ([_P, i32, _P, i32, i32, ctypes.c_float, i32, _P, _P], i32),
            "neb_get_stats": ([_P, ctypes.POINTER(Stats)], i32),
            "neb_get_path_records": ([_P, _P, i64], i32),
            "neb_get_octree": ([_P, _P, i32, _P], i32),
            "neb_get_scene_octree": ([_P, i32, _P, i32, _P], i32),
            "neb_profile_kernels": ([_P, i32], i32),
            "neb_get_kernel_profile": ([_P, ctypes.POINTER(KernelTime), i32, ctypes.POINTER(i32)], i32),
            "neb_reset": ([_P], i32),
            "neb_destroy": ([_P], None),
            "neb_status_string": ([i32], ctypes.c_char_p),
            "neb_last_error": ([], ctypes.c_char_p),
            "neb_configure_mlp": ([_P, ctypes.POINTER(MlpParams)], i32),
            "neb_get_mlp_status": ([_P, ctypes.POINTER(MlpStatus)], i32),
            "neb_get_mlp_weights": ([_P, _P], i32),
            "neb_set_mlp_model": ([_P, _P, ctypes.c_float, ctypes.c_float], i32),
            "neb_get_mlp_gates": ([_P, _P, _P, _P], i32),
            "neb_mlp_create": ([_P, ctypes.c_uint32, i32, ctypes.POINTER(_P)], i32),
            "neb_mlp_set_normalization": ([_P, ctypes.c_float, ctypes.c_float, _P], i32),
            "neb_mlp_infer": ([_P, _P, _P, i32, _P, _P], i32),
            "neb_mlp_gradient": ([_P, _P, _P, _P, i32, _P, ctypes.POINTER(ctypes.c_float), _P], i32),
            "neb_mlp_train_step": ([_P, _P, _P, _P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, _P], i32),
            "neb_mlp_get_params": ([_P, _P], i32),
            "neb_mlp_destroy": ([_P], None),
            "neb_octree_create": ([_P, _P, i32, ctypes.POINTER(_P)], i32),
            "neb_octree_set_iteration": ([_P, i32], i32),
            "neb_octree_increment": ([_P, _P, i32, i32, _P], i32),
            "neb_octree_density": ([_P, _P, _P, i32, i32, _P, _P], i32),
            "neb_octree_clear_counters": ([_P, _P], i32),
            "neb_octree_export": ([_P, _P, i32, _P, _P], i32),
            "neb_octree_destroy": ([_P], None),
            "neb_atomic_probe": ([_P, i32, i32, i32, i32, i32, _P, _P], i32),
            "neb_gather_probe": ([_P, ctypes.c_int64, i32, i32, i32, _P, _P], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status):
    if status != NEB_OK:
        L = lib()
        raise NebError(f"{L.neb_status_string(status).decode()}: {L.neb_last_error().decode()}")


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _dev_ptr(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise NebError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def make_params(scene, density_mode=DENSITY_OCTREE_ROBUST, flags=0, rho0=0.0, cam_weight=0.0, **over):
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
    p.flags = flags
    p.spp = over.get("spp", 0)
    p.light_photons = over.get("light_photons", 0)
    p.density_radius = over.get("density_radius", 0.0)
    p.knn_k = over.get("knn_k", 8)
    p.nee_radius = over.get("nee_radius", 0.0)
    return p


def point_density(points, queries, mode, radius, k=8, out=None, stream=None):
    """Fixed-radius (DENSITY_RADIUS) or k-nearest-neighbour (DENSITY_KNN)
    density of the query points over the point set, per unit area
    (neb_point_density).  points (n, 3) and queries (m, 3): float32 device
    tensors; returns an (m,) float32 device tensor."""
    import torch
    assert points.dtype == torch.float32 and queries.dtype == torch.float32
    assert points.is_contiguous() and queries.is_contiguous()
    m = queries.shape[0]
    if out is None:
        out = torch.empty(m, dtype=torch.float32, device=queries.device)
    _check(lib().neb_point_density(_dev_ptr(points) if points.numel() else None, points.shape[0],
                                   _dev_ptr(queries), m, int(mode), float(radius), int(k), _dev_ptr(out),
                                   _stream(stream)))
    return out


def point_density_noalloc(points, queries, mode, radius, k, out, stream=None):
    """neb_point_density_noalloc: as point_density, into the caller's `out`
    (an (m,) float32 device tensor), enqueued on `stream` without any
    device allocation; at most 2^19 points."""
    import torch
    assert points.dtype == torch.float32 and queries.dtype == torch.float32 and out.dtype == torch.float32
    _check(lib().neb_point_density_noalloc(_dev_ptr(points) if points.numel() else None, points.shape[0],
                                           _dev_ptr(queries), queries.shape[0], int(mode), float(radius), int(k),
                                           _dev_ptr(out), _stream(stream)))
    return out


def _scene_arrays(scene):
    return [np.ascontiguousarray(scene.vertices, np.float32), np.ascontiguousarray(scene.tris, np.int32),
            np.ascontiguousarray(scene.tri_mat, np.int32), np.ascontiguousarray(scene.materials),
            np.ascontiguousarray(scene.point_lights), np.ascontiguousarray(scene.camera)]


class BatchRenderer:
    """A context rendering several scenes together (neb_create_batch); every
    launch covers all of them.  Per-scene settings come from each scene
    object (its image size, path length, octree capacity, merge radius, seed,
    scene id and spp) unless overridden by `per_scene` dicts."""

    def __init__(self, scenes, density_mode=DENSITY_OCTREE_ROBUST, flags=0, rho0=0.0, cam_weight=0.0,
                 per_scene=None, spp=None):
        self.scenes = list(scenes)
        n = len(self.scenes)
        per_scene = per_scene or [{} for _ in range(n)]
        arr = (Params * n)()
        for i, sc in enumerate(self.scenes):
            over = dict(per_scene[i])
            if spp is not None:
                over.setdefault("spp", spp[i] if hasattr(spp, "__len__") else spp)
            arr[i] = make_params(sc, density_mode, flags, rho0, cam_weight, **over)
        self.params_list = [arr[i] for i in range(n)]
        h = _P()
        _check(lib().neb_create_batch(arr, n, ctypes.byref(h)))
        self.h = h
        for i, sc in enumerate(self.scenes):
            self._set(i, sc)

    def _set(self, i, scene):
        v, t, m, mats, pl, cam = _scene_arrays(scene)
        _check(lib().neb_set_batch_scene(self.h, i, _np_ptr(v), v.shape[0], _np_ptr(t), _np_ptr(m), t.shape[0],
                                         _np_ptr(mats), mats.shape[0], _np_ptr(pl) if len(pl) else None,
                                         pl.shape[0], _np_ptr(cam)))

    def close(self):
        if getattr(self, "h", None):
            lib().neb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def render(self, n_iterations, stream=None):
        _check(lib().neb_render(self.h, int(n_iterations), _stream(stream)))

    def use_graph(self, mode=1):
        """0: eager launches, 1 (or True): one graph per iteration, 2: one
        graph per render call."""
        _check(lib().neb_use_graph(self.h, int(mode)))

    def autotune(self, trial_iterations=2, stream=None):
        cfg = LaunchConfig()
        _check(lib().neb_autotune(self.h, int(trial_iterations), _stream(stream), ctypes.byref(cfg)))
        return cfg.as_dict()

    def set_launch_config(self, bvh_stack, trace_blocks_per_cu, photon_blocks_per_cu, photon_order=0,
                          nee_blocks_per_cu=-1, concurrent=1):
        cfg = LaunchConfig(bvh_stack, trace_blocks_per_cu, nee_blocks_per_cu, photon_blocks_per_cu, photon_order,
                           concurrent)
        _check(lib().neb_set_launch_config(self.h, ctypes.byref(cfg)))

    def launch_config(self):
        cfg = LaunchConfig()
        _check(lib().neb_get_launch_config(self.h, ctypes.byref(cfg)))
        return cfg.as_dict()

    def image(self, scene=0, out=None, stream=None):
        """Mean radiance of one scene: a (H, W, 3) float32 device tensor
        (written into `out` if given)."""
        import torch
        P = self.params_list[scene]
        if out is None:
            out = torch.empty((P.height, P.width, 3), dtype=torch.float32, device="cuda")
        _check(lib().neb_get_scene_image(self.h, int(scene), _dev_ptr(out), 1, _stream(stream)))
        return out

    def image_host(self, scene=0):
        P = self.params_list[scene]
        out = np.zeros((P.height, P.width, 3), np.float32)
        _check(lib().neb_get_scene_image(self.h, int(scene), _np_ptr(out), 0, None))
        return out

    def technique_images_host(self, scene=0):
        """Mean radiance per technique: random hits e, NEE E, NEB photons P
        and conventional light photons LP (zero without light photons)."""
        P = self.params_list[scene]
        e, E, Pi, LP = (np.zeros((P.height, P.width, 3), np.float32) for _ in range(4))
        _check(lib().neb_get_scene_technique_images(self.h, int(scene), _np_ptr(e), _np_ptr(E), _np_ptr(Pi), 0,
                                                    None))
        _check(lib().neb_get_scene_light_photon_image(self.h, int(scene), _np_ptr(LP), 0, None))
        return {"e": e, "E": E, "P": Pi, "LP": LP}

    def stats(self):
        s = Stats()
        _check(lib().neb_get_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def records(self):
        """Path records of the first iteration: (pixels over all scenes,
        longest path length)."""
        npix = sum(P.width * P.height for P in self.params_list)
        L = max(P.max_path_len for P in self.params_list)
        out = np.zeros(npix * L, RECORD_DTYPE)
        _check(lib().neb_get_path_records(self.h, _np_ptr(out), out.size))
        return out.reshape(npix, L)

    def octree(self, scene=0):
        info = np.zeros(8, np.int64)
        _check(lib().neb_get_scene_octree(self.h, int(scene), None, 0, _np_ptr(info)))
        nodes = np.zeros(int(info[0]), np.int32)
        _check(lib().neb_get_scene_octree(self.h, int(scene), _np_ptr(nodes), nodes.size, _np_ptr(info)))
        return nodes, dict(zip(OCT_INFO_KEYS, (int(x) for x in info)))

    def query_density(self, pos, nrm, stream=None):
        """Scene 0's octree.  pos, nrm: (n, 3) float32 device tensors -> (n,)
        densities."""
        import torch
        out = torch.empty(pos.shape[0], dtype=torch.float32, device=pos.device)
        _check(lib().neb_query_density(self.h, _dev_ptr(pos), _dev_ptr(nrm), pos.shape[0], _dev_ptr(out), 1,
                                       _stream(stream)))
        return out

    def profile_kernels(self, enable=True):
        _check(lib().neb_profile_kernels(self.h, int(enable)))

    def kernel_profile(self):
        arr = (KernelTime * 32)()
        n = ctypes.c_int32()
        _check(lib().neb_get_kernel_profile(self.h, arr, 32, ctypes.byref(n)))
        return {arr[i].name.decode(): {"launches": int(arr[i].launches), "total_ms": float(arr[i].total_ms)}
                for i in range(n.value)}

    def reset(self):
        _check(lib().neb_reset(self.h))

    def configure_mlp(self, **kw):
        """Learned-density settings (NEB_DENSITY_MLP contexts); restarts."""
        d = dict(MLP_DEFAULTS)
        d.update(kw)
        p = MlpParams(**d)
        _check(lib().neb_configure_mlp(self.h, ctypes.byref(p)))

    def mlp_status(self):
        st = MlpStatus()
        _check(lib().neb_get_mlp_status(self.h, ctypes.byref(st)))
        return st.as_dict()

    def set_mlp_model(self, params, mu, sigma):
        """Use the given model (NEB_MLP_PARAMS floats; log rho = mu + sigma y)
        instead of the seeded initial weights; None returns to those.
        Restarts the context."""
        if params is None:
            _check(lib().neb_set_mlp_model(self.h, None, 0.0, 1.0))
            return
        w = np.ascontiguousarray(params, np.float32)
        assert w.size == MLP_PARAMS
        _check(lib().neb_set_mlp_model(self.h, _np_ptr(w), float(mu), float(sigma)))

    def mlp_gates(self):
        """Region gates and probe tallies, each (32, 32, 32) int32 indexed
        [z, y, x] (region x + 32 (y + 32 z))."""
        g, t, b = (np.zeros(32 ** 3, np.int32) for _ in range(3))
        _check(lib().neb_get_mlp_gates(self.h, _np_ptr(g), _np_ptr(t), _np_ptr(b)))
        return {"gate": g.reshape(32, 32, 32), "probes": t.reshape(32, 32, 32), "bad": b.reshape(32, 32, 32)}

    def mlp_weights(self):
        out = np.zeros(MLP_PARAMS, np.float32)
        _check(lib().neb_get_mlp_weights(self.h, _np_ptr(out)))
        return out


class Renderer(BatchRenderer):
    """One rendering context of one scene on the current device (a batch of
    one; progressive: every iteration counts unless spp is given)."""

    def __init__(self, scene, density_mode=DENSITY_OCTREE_ROBUST, flags=0, rho0=0.0, cam_weight=0.0, **over):
        self.params = make_params(scene, density_mode, flags, rho0, cam_weight, **over)
        self.params_list = [self.params]
        self.scenes = [scene]
        self.scene = scene
        h = _P()
        _check(lib().neb_create(ctypes.byref(self.params), ctypes.byref(h)))
        self.h = h
        v, t, m, mats, pl, cam = _scene_arrays(scene)
        _check(lib().neb_set_scene(self.h, _np_ptr(v), v.shape[0], _np_ptr(t), _np_ptr(m), t.shape[0],
                                   _np_ptr(mats), mats.shape[0], _np_ptr(pl) if len(pl) else None, pl.shape[0],
                                   _np_ptr(cam)))

    def records(self):
        n = self.params.width * self.params.height * self.params.max_path_len
        out = np.zeros(n, RECORD_DTYPE)
        _check(lib().neb_get_path_records(self.h, _np_ptr(out), n))
        return out.reshape(self.params.width * self.params.height, self.params.max_path_len)


def atomic_probe(words, n_words, stride, blocks, ops, kind, sink, stream=None):
    """neb_atomic_probe on int32 device tensors `words` (>= n_words * stride)
    and `sink` (>= blocks * 256)."""
    assert words.numel() >= n_words * stride and sink.numel() >= blocks * 256
    _check(lib().neb_atomic_probe(_dev_ptr(words), int(n_words), int(stride), int(blocks), int(ops), int(kind),
                                  _dev_ptr(sink), _stream(stream)))


def gather_probe(buf, width, blocks, ops, sink, stream=None):
    """neb_gather_probe on a float32 device tensor `buf` (its size in 16-byte
    words is n_words) and `sink` (>= blocks * 256 floats)."""
    assert buf.numel() % 4 == 0 and sink.numel() >= blocks * 256
    _check(lib().neb_gather_probe(_dev_ptr(buf), int(buf.numel() // 4), int(width), int(blocks), int(ops),
                                  _dev_ptr(sink), _stream(stream)))


class Mlp:
    """Standalone learned-density model on the current device."""

    def __init__(self, init=None, seed=1, max_batch=65536):
        h = _P()
        w = None if init is None else np.ascontiguousarray(init, np.float32)
        if w is not None and w.size != MLP_PARAMS:
            raise NebError("init must hold MLP_PARAMS values")
        _check(lib().neb_mlp_create(_np_ptr(w) if w is not None else None, int(seed), int(max_batch),
                                    ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().neb_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_normalization(self, mu, sigma, stream=None):
        _check(lib().neb_mlp_set_normalization(self.h, float(mu), float(sigma), _stream(stream)))

    def infer(self, q, nrm, stream=None):
        import torch
        out = torch.empty(q.shape[0], dtype=torch.float32, device=q.device)
        _check(lib().neb_mlp_infer(self.h, _dev_ptr(q), _dev_ptr(nrm), q.shape[0], _dev_ptr(out), _stream(stream)))
        return out

    def gradient(self, q, nrm, log_rho, stream=None):
        import torch
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=q.device)
        loss = ctypes.c_float()
        _check(lib().neb_mlp_gradient(self.h, _dev_ptr(q), _dev_ptr(nrm), _dev_ptr(log_rho), q.shape[0],
                                      _dev_ptr(g), ctypes.byref(loss), _stream(stream)))
        return g, float(loss.value)

    def train_step(self, q, nrm, log_rho, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib().neb_mlp_train_step(self.h, _dev_ptr(q), _dev_ptr(nrm), _dev_ptr(log_rho), q.shape[0],
                                        float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))

    def params(self):
        out = np.zeros(MLP_PARAMS, np.float32)
        _check(lib().neb_mlp_get_params(self.h, _np_ptr(out)))
        return out


class DeviceOctree:
    """The density octree of Appendix B on the GPU (batched calls)."""

    def __init__(self, smin, smax, capacity):
        a = np.ascontiguousarray(smin, np.float32)
        b = np.ascontiguousarray(smax, np.float32)
        h = _P()
        _check(lib().neb_octree_create(_np_ptr(a), _np_ptr(b), int(capacity), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().neb_octree_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_iteration(self, it):
        _check(lib().neb_octree_set_iteration(self.h, int(it)))

    def increment(self, pos, single_thread=False, stream=None):
        _check(lib().neb_octree_increment(self.h, _dev_ptr(pos), pos.shape[0], int(single_thread), _stream(stream)))

    def density(self, pos, nrm, robust=True, stream=None):
        import torch
        out = torch.empty(pos.shape[0], dtype=torch.float32, device=pos.device)
        _check(lib().neb_octree_density(self.h, _dev_ptr(pos), _dev_ptr(nrm), pos.shape[0], int(robust),
                                        _dev_ptr(out), _stream(stream)))
        return out

    def clear_counters(self, stream=None):
        _check(lib().neb_octree_clear_counters(self.h, _stream(stream)))

    def export(self, stream=None):
        info = np.zeros(8, np.int64)
        _check(lib().neb_octree_export(self.h, None, 0, _np_ptr(info), _stream(stream)))
        nodes = np.zeros(int(info[0]), np.int32)
        _check(lib().neb_octree_export(self.h, _np_ptr(nodes), nodes.size, _np_ptr(info), _stream(stream)))
        return nodes, dict(zip(OCT_INFO_KEYS, (int(x) for x in info)))
