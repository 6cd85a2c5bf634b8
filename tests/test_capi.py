"""The C-ABI library loads on the CPU and exports every function that
include/neb.h declares (no compute call is made without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "neb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:neb_status|void|const char\*)\s+(neb_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("neb_create", "neb_set_scene", "neb_render", "neb_get_image", "neb_query_density",
                 "neb_octree_create", "neb_octree_increment", "neb_octree_density", "neb_octree_export"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1909_00573_amd import neb
    if not os.path.exists(neb.LIB_PATH):
        pytest.skip("libneb.so not built")
    L = neb.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert missing == []
    assert sorted(neb.EXPORTS) == _declared()
    assert L.neb_status_string(-1) == b"invalid argument"


def test_invalid_arguments_are_rejected_without_a_device():
    """Argument checks happen before any HIP call."""
    import ctypes
    from paper_1909_00573_amd import neb
    if not os.path.exists(neb.LIB_PATH):
        pytest.skip("libneb.so not built")
    L = neb.lib()
    p = neb.Params()
    p.width, p.height, p.max_path_len, p.octree_capacity, p.merge_radius = 0, 8, 4, 64, 0.01
    h = ctypes.c_void_p()
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1
    p.width, p.max_path_len = 8, 99
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1
    p.max_path_len, p.merge_radius = 4, -1.0
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1
    assert L.neb_render(None, 1, None) == -1
    lo = (ctypes.c_float * 3)(0, 0, 0)
    assert L.neb_octree_create(lo, lo, 16, ctypes.byref(h)) == -1     # flat bounds
    # batch, graph and tuning entry points check their arguments first
    one = (neb.Params * 2)()
    for q in one:
        q.width, q.height, q.max_path_len, q.octree_capacity, q.merge_radius = 8, 8, 4, 64, 0.01
    assert L.neb_create_batch(one, 0, ctypes.byref(h)) == -1
    assert L.neb_create_batch(one, 257, ctypes.byref(h)) == -1
    one[1].density_mode = 3
    assert L.neb_create_batch(one, 2, ctypes.byref(h)) == -1          # mixed density modes
    one[1].density_mode = 0
    one[1].spp = -1
    assert L.neb_create_batch(one, 2, ctypes.byref(h)) == -1
    assert L.neb_use_graph(None, 1) == -1
    assert L.neb_autotune(None, 1, None, None) == -1
    assert L.neb_set_launch_config(None, None) == -1
    assert L.neb_get_scene_image(None, 0, None, 0, None) == -1
    assert L.neb_set_batch_scene(None, 0, None, 0, None, None, 0, None, 0, None, 0, None) == -1
    mh = ctypes.c_void_p()
    assert L.neb_mlp_create(None, 1, 0, ctypes.byref(mh)) == -1          # max_batch < 1
    assert L.neb_mlp_infer(None, None, None, 1, None, None) == -1
    assert L.neb_configure_mlp(None, None) == -1
    one[1].spp = 0
    one[0].density_mode = one[1].density_mode = 2
    assert L.neb_create_batch(one, 2, ctypes.byref(h)) == -1          # learned density: one scene only


def test_light_photon_and_density_provider_arguments_without_a_device():
    """Light photons, the alternative density providers and the point-set
    density entry point validate their arguments before any HIP call."""
    import ctypes
    from paper_1909_00573_amd import neb
    if not os.path.exists(neb.LIB_PATH):
        pytest.skip("libneb.so not built")
    L = neb.lib()
    h = ctypes.c_void_p()
    p = neb.Params()
    p.width, p.height, p.max_path_len, p.octree_capacity, p.merge_radius = 8, 8, 4, 64, 0.01
    p.light_photons = -1
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1
    p.light_photons = (1 << 26) + 1
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1
    p.light_photons, p.density_mode = 64, 2
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1          # light photons with the learned density
    p.light_photons = 0
    for mode in (4, 5):
        p.density_mode, p.density_radius, p.knn_k = mode, 0.0, 8
        assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1      # radius must be > 0
    p.density_mode, p.density_radius, p.knn_k = 5, 0.1, 17
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1          # k above 16
    p.density_mode = 6
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1          # unknown mode
    # neb_point_density: mode, radius, k and sizes; an empty query set is a no-op
    assert L.neb_point_density(None, 0, None, 1, 3, ctypes.c_float(0.1), 4, None, None) == -1
    assert L.neb_point_density(None, 0, None, 1, 4, ctypes.c_float(0.0), 4, None, None) == -1
    assert L.neb_point_density(None, 0, None, 1, 5, ctypes.c_float(0.1), 0, None, None) == -1
    assert L.neb_point_density(None, -1, None, 1, 4, ctypes.c_float(0.1), 4, None, None) == -1
    assert L.neb_point_density(None, 5, None, 0, 4, ctypes.c_float(0.1), 4, None, None) == 0
    assert L.neb_point_density(None, 5, None, 3, 4, ctypes.c_float(0.1), 4, None, None) == -1   # null pointers
    assert L.neb_get_scene_light_photon_image(None, 0, None, 0, None) == -1


def test_recycling_arguments_without_a_device():
    import ctypes
    from paper_1909_00573_amd import neb
    if not os.path.exists(neb.LIB_PATH):
        pytest.skip("libneb.so not built")
    L = neb.lib()
    h = ctypes.c_void_p()
    p = neb.Params()
    p.width, p.height, p.max_path_len, p.octree_capacity, p.merge_radius = 8, 8, 4, 64, 0.01
    p.nee_radius = -0.1
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1
    p.nee_radius, p.light_photons = 0.1, 16
    assert L.neb_create(ctypes.byref(p), ctypes.byref(h)) == -1          # not with light photons
    two = (neb.Params * 2)()
    for q in two:
        q.width, q.height, q.max_path_len, q.octree_capacity, q.merge_radius = 8, 8, 4, 64, 0.01
    two[0].nee_radius = 0.1
    assert L.neb_create_batch(two, 2, ctypes.byref(h)) == -1           # on for one scene only
