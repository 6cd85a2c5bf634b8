"""Concurrent launches (the default: NEE's shadow rays and the merge grid on
a second stream beside the octree deposits and the density, each bounce's
merges beside the next bounce's closest hits) against every launch on one
stream.  The two orders of execution must give the same estimator: with
the deterministic single-thread octree the trees, the work statistics and
the per-technique images agree up to the order of floating-point
additions, for plain NEB, with light photons, with NEE recycling and for a
batch of scenes; eager launches and graph replays (of one iteration, or
of a whole call) agree too.  With the
second stream on, each iteration of a call but the last also runs the next
iteration's camera pass on a third stream (from the iteration's start, or
after the deposits when single-thread deposits share their slots with it);
with the analytic density, which needs no octree, the parallel deposits
are checked too, and so is splitting the iterations over several calls."""
import numpy as np
import pytest

from neb_inputs import tiny_box, box_room

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def neb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_00573_amd import neb as N
    N.lib()
    return N


def _close(a, b, rtol=2e-4):
    a = a.astype(np.float64)
    b = b.astype(np.float64)
    return np.all(np.abs(a - b) <= rtol * np.abs(a) + 1e-6 * max(np.abs(a).max(), 1e-30))


def _pair(neb, make, n_iter, graph=False, order=None):
    out = []
    for conc in (1, 0):
        R = make()
        cfg = R.launch_config()
        R.set_launch_config(cfg["bvh_stack"], cfg["trace_blocks_per_cu"], cfg["photon_blocks_per_cu"],
                            cfg["photon_order"] if order is None else order, cfg["nee_blocks_per_cu"],
                            concurrent=conc)
        if graph:
            R.use_graph(True)
        R.render(n_iter)
        out.append((R.technique_images_host(), R.stats(), R.octree()[0]))
        R.close()
    return out


@pytest.mark.parametrize("kw", [{}, {"light_photons": 4096}, {"nee_radius": 0.03}])
def test_concurrent_equals_serial(neb, kw):
    sc = tiny_box(width=48, height=40, max_path_len=6)
    (ta, sa, oa), (tb, sb, ob) = _pair(neb, lambda: neb.Renderer(sc, flags=neb.FLAG_SINGLE_THREAD_OCTREE, **kw), 4)
    assert np.array_equal(oa, ob)
    for k in ("vertices", "photons", "photon_segments", "merges", "candidates", "shadow_rays", "nee_visible",
              "light_photons"):
        assert sa[k] == sb[k], k
    for t in ("e", "E", "P", "LP"):
        assert _close(ta[t], tb[t]), t
    assert sa["merges"] > 0


@pytest.mark.parametrize("order", [0, 1])
def test_concurrent_equals_serial_photon_orders(neb, order):
    """Merges in queue order and in Morton-bin order, each with the
    bounce's merges beside the next bounce's closest hits: the shared order
    array is rewritten only after the merges of the bounce before."""
    sc = tiny_box(width=48, height=40, max_path_len=8)
    (ta, sa, oa), (tb, sb, ob) = _pair(
        neb, lambda: neb.Renderer(sc, flags=neb.FLAG_SINGLE_THREAD_OCTREE, light_photons=4096), 4, order=order)
    assert np.array_equal(oa, ob)
    for k in ("photons", "photon_segments", "merges", "candidates", "light_photons"):
        assert sa[k] == sb[k], k
    for t in ("e", "E", "P", "LP"):
        assert _close(ta[t], tb[t]), t


def test_concurrent_equals_serial_batch_and_graph(neb):
    scenes = [box_room(n_tris=2000, n_lights=3, res=64, seed=5 + k, scene_id=k) for k in range(3)]
    make = lambda: neb.BatchRenderer(scenes, flags=neb.FLAG_SINGLE_THREAD_OCTREE)
    for graph in (0, 1, 2):
        (ta, sa), (tb, sb) = _pair_batch(neb, make, 3, graph)
        assert sa["merges"] == sb["merges"] and sa["vertices"] == sb["vertices"]
        for s in range(len(scenes)):
            for t in ("e", "E", "P"):
                assert _close(ta[s][t], tb[s][t]), (graph, s, t)


def _pair_batch(neb, make, n_iter, graph):
    out = []
    for conc in (1, 0):
        B = make()
        cfg = B.launch_config()
        B.set_launch_config(cfg["bvh_stack"], cfg["trace_blocks_per_cu"], cfg["photon_blocks_per_cu"],
                            cfg["photon_order"], cfg["nee_blocks_per_cu"], concurrent=conc)
        B.use_graph(graph)
        B.render(n_iter)
        out.append(([B.technique_images_host(s) for s in range(len(B.scenes))], B.stats()))
        B.close()
    return out


def _analytic(neb, conc, graph, calls):
    sc = tiny_box(width=48, height=40, max_path_len=6)
    R = neb.Renderer(sc, density_mode=neb.DENSITY_ANALYTIC, rho0=3000.0, cam_weight=1.0)
    cfg = R.launch_config()
    R.set_launch_config(cfg["bvh_stack"], cfg["trace_blocks_per_cu"], cfg["photon_blocks_per_cu"],
                        cfg["photon_order"], cfg["nee_blocks_per_cu"], concurrent=conc)
    R.use_graph(graph)
    for n in calls:
        R.render(n)
    out = (R.technique_images_host(), R.stats())
    R.close()
    return out


@pytest.mark.parametrize("graph", [0, 1, 2])
def test_next_camera_pass_beside_iteration(neb, graph):
    ta, sa = _analytic(neb, 1, graph, [5])
    tb, sb = _analytic(neb, 0, graph, [5])
    tc, sc_ = _analytic(neb, 1, graph, [2, 1, 2])
    for s_ in (sb, sc_):
        for k in ("iterations", "camera_rays", "vertices", "photons", "photon_segments", "merges", "candidates",
                  "shadow_rays", "nee_visible"):
            assert sa[k] == s_[k], k
    for t in ("e", "E", "P"):
        assert _close(ta[t], tb[t]), t
        assert _close(ta[t], tc[t]), t
    assert sa["merges"] > 0 and sa["iterations"] == 5


def test_concurrent_equals_serial_learned_density(neb):
    """The learned density (a given model, no training steps) with the next
    iteration's camera pass on the third stream, against every launch on
    one stream: same probes, gates, fallbacks and images."""
    from oracle import mlp as M
    theta = M.init_params(7).astype(np.float32)
    sc = tiny_box(width=48, height=40, max_path_len=6)
    out = []
    for conc in (1, 0):
        R = neb.Renderer(sc, density_mode=neb.DENSITY_MLP, flags=neb.FLAG_SINGLE_THREAD_OCTREE)
        cfg = R.launch_config()
        R.set_launch_config(cfg["bvh_stack"], cfg["trace_blocks_per_cu"], cfg["photon_blocks_per_cu"],
                            cfg["photon_order"], cfg["nee_blocks_per_cu"], concurrent=conc)
        R.configure_mlp(train_iterations=2, steps_per_iteration=0, probe_every=2, probes=500, max_rel_error=0.5)
        R.set_mlp_model(theta, np.log(3000.0), 0.3)
        R.render(7)
        out.append((R.technique_images_host(), R.stats(), R.mlp_status(), R.mlp_gates()))
        R.close()
    (ta, sa, ma, ga), (tb, sb, mb, gb) = out
    for k in ("vertices", "photons", "photon_segments", "merges", "nee_visible"):
        assert sa[k] == sb[k], k
    for k in ("probes", "probes_bad", "regions_probed", "regions_disabled", "fallback_queries", "probes_served"):
        assert ma[k] == mb[k], k
    assert ma["regions_disabled"] > 0 and ma["fallback_queries"] > 0 and ma["probes_served"] > 0
    for k in ("gate", "probes", "bad"):
        assert np.array_equal(ga[k], gb[k]), k
    for t in ("e", "E", "P"):
        assert _close(ta[t], tb[t]), t


def test_graph_mode_is_checked(neb):
    """Graph modes are 0 (eager), 1 (one graph per iteration) and 2 (one
    graph per call); another mode is refused and leaves the context as it
    was."""
    sc = tiny_box(width=16, height=16, max_path_len=3)
    R = neb.Renderer(sc, density_mode=neb.DENSITY_ANALYTIC, rho0=3000.0, cam_weight=1.0)
    for bad in (-1, 3):
        with pytest.raises(neb.NebError):
            R.use_graph(bad)
    R.use_graph(2)
    R.render(2)
    assert R.stats()["iterations"] == 2
    R.close()
