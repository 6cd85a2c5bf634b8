"""Batched rendering, captured iterations and launch-shape tuning on the GPU.

A batch renders several scenes of different sizes, path lengths and spp in
one launch per stage.  Because every scene draws its random numbers with
its own key and scene-local pixel numbers, a scene renders in a batch the
same estimator as alone:
- with the analytic density, every recorded view path is bit-identical
  to the scene rendered alone, and the images agree up to the order of the
  floating-point image additions;
- with the single-thread octree, every scene's octree node array is
  identical to the one it builds alone;
- with the concurrent octree, every scene's ledger is conserved;
- one batched scene matches the FP64 oracle.
A captured iteration, or a captured call of several iterations, replayed
as a HIP graph reproduces the eager launches after every replay, and the autotuner's launch shapes change the
speed, not the results.
"""
import numpy as np
import pytest

from neb_inputs import tiny_box, box_room

pytestmark = pytest.mark.gpu

RHO0 = 3000.0


@pytest.fixture(scope="module")
def neb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_00573_amd import neb as N
    N.lib()
    return N


def _scenes():
    a = tiny_box(width=48, height=40, max_path_len=5, seed=1)
    b = tiny_box(width=64, height=64, max_path_len=4, seed=9).with_settings(scene_id=5)
    c = box_room(n_tris=3000, n_lights=4, res=72, seed=4, scene_id=2)
    return [a, b, c], [3, 0, 2]


@pytest.fixture(scope="module")
def batch_scenes():
    return _scenes()


def close(a, b, rtol=1e-4):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    tol = rtol * np.abs(b) + 1e-6 * max(np.abs(b).max(), 1e-30)
    return bool(np.all(np.abs(a - b) <= tol))


def _offsets(scenes):
    pix = np.cumsum([0] + [s.width * s.height for s in scenes])
    tri = np.cumsum([0] + [s.n_tris for s in scenes])
    mat = np.cumsum([0] + [len(s.materials) for s in scenes])
    return pix, tri, mat


def test_batched_paths_and_images_equal_alone(neb, batch_scenes):
    scenes, spp = batch_scenes
    n_iter = 4
    B = neb.BatchRenderer(scenes, density_mode=neb.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0,
                          flags=neb.FLAG_RECORD_PATHS, spp=spp)
    B.render(n_iter)
    rb = B.records()
    pix, tri, mat = _offsets(scenes)
    total_vertices = 0
    for s, sc in enumerate(scenes):
        A = neb.Renderer(sc, density_mode=neb.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0,
                         flags=neb.FLAG_RECORD_PATHS, spp=spp[s])
        A.render(n_iter)
        ra = A.records()
        part = rb[pix[s]:pix[s + 1], :sc.max_path_len]
        assert np.array_equal(part["type"], ra["type"]), s
        live = (ra["type"] >= 1) & (ra["type"] <= 4)
        assert np.array_equal(part["pos"][live], ra["pos"][live]), s
        assert np.array_equal(part["mat"][live] - mat[s], ra["mat"][live]), s
        assert np.array_equal(part["prim"][live] - tri[s], ra["prim"][live]), s
        # rows past the scene's path length are never written
        assert np.all(rb[pix[s]:pix[s + 1], sc.max_path_len:]["type"] == 0)
        tb, ta = B.technique_images_host(s), A.technique_images_host()
        for t in ("e", "E", "P"):
            assert close(tb[t], ta[t]), (s, t)
        assert close(B.image_host(s), A.image_host()), s
        total_vertices += A.stats()["vertices"]
        A.close()
    st = B.stats()
    assert st["vertices"] == total_vertices
    assert st["iterations"] == n_iter
    # every scene took part in min(spp, n_iter) iterations
    assert st["paths"] == sum(sc.width * sc.height * (min(p, n_iter) if p else n_iter)
                              for sc, p in zip(scenes, spp))
    B.close()


def test_batched_single_thread_octrees_equal_alone(neb, batch_scenes):
    scenes, spp = batch_scenes
    n_iter = 3
    B = neb.BatchRenderer(scenes, flags=neb.FLAG_SINGLE_THREAD_OCTREE, spp=spp)
    B.render(n_iter)
    root = 0
    for s, sc in enumerate(scenes):
        A = neb.Renderer(sc, flags=neb.FLAG_SINGLE_THREAD_OCTREE, spp=spp[s])
        A.render(n_iter)
        nb, ib = B.octree(s)
        na, ia = A.octree()
        local = np.where(nb < 0, nb + root, nb)
        assert np.array_equal(local, na), s
        assert ib == ia, s
        assert ib["ledger"] == ib["deposits"] > 0
        tb, ta = B.technique_images_host(s), A.technique_images_host()
        for t in ("e", "E", "P"):
            assert close(tb[t], ta[t], rtol=1e-3), (s, t)
        root += ib["capacity"]
        A.close()
    B.close()


def test_batched_concurrent_octree_ledgers(neb, batch_scenes):
    scenes, spp = batch_scenes
    B = neb.BatchRenderer(scenes, spp=spp)
    B.render(4)
    st = B.stats()
    dep = 0
    for s in range(len(scenes)):
        _, info = B.octree(s)
        assert info["ledger"] == info["deposits"], s
        assert info["lost"] == 0
        dep += info["deposits"]
    assert dep + st["oct_rejected"] == st["vertices"]
    assert st["oct_ledger"] == st["oct_deposits"] == dep
    B.close()


def test_batched_scene_matches_oracle(neb, oracle, batch_scenes):
    scenes, spp = batch_scenes
    B = neb.BatchRenderer(scenes, density_mode=neb.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0, spp=spp)
    B.render(4)
    img = B.image_host(0).astype(np.float64)
    o = oracle.render(scenes[0], n_iter=spp[0], density_mode=oracle.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0)
    err = float(np.sqrt(np.mean((img - o["mean"]) ** 2)) / np.mean(o["mean"]))
    assert err < 0.01, err
    B.close()


@pytest.mark.parametrize("mode,per_call", [(1, 1), (2, 2)])
def test_graph_replays_match_eager_launches(neb, batch_scenes, mode, per_call):
    """Every replay of the captured iteration (mode 1) or of the captured
    two-iteration call (mode 2: the next camera pass forked inside the
    graph) is checked against the eager context, with eager device work and
    synchronisations between replays."""
    import torch
    scenes, spp = batch_scenes
    E = neb.BatchRenderer(scenes, flags=neb.FLAG_SINGLE_THREAD_OCTREE, spp=spp)
    G = neb.BatchRenderer(scenes, flags=neb.FLAG_SINGLE_THREAD_OCTREE, spp=spp)
    G.use_graph(mode)
    for it in range(1, 5):
        E.render(per_call)
        G.render(per_call)
        x = torch.randn(1 << 16, device="cuda")
        float(x.square().sum())  # unrelated eager work between replays
        torch.cuda.synchronize()
        se, sg = E.stats(), G.stats()
        for k in ("iterations", "paths", "vertices", "photons", "merges", "events", "oct_deposits", "oct_ledger"):
            assert se[k] == sg[k], (it, k)
        for s in range(len(scenes)):
            ne, ie = E.octree(s)
            ng, ig = G.octree(s)
            assert np.array_equal(ne, ng), (it, s)
            assert close(E.image_host(s), G.image_host(s), rtol=1e-3), (it, s)
    E.close()
    G.close()


def test_autotune_changes_speed_not_results(neb, batch_scenes):
    scenes, spp = batch_scenes
    T = neb.BatchRenderer(scenes, flags=neb.FLAG_SINGLE_THREAD_OCTREE, spp=spp)
    cfg = T.autotune(1)
    assert cfg["bvh_stack"] in (32, 48, 64)
    assert 0 <= cfg["trace_blocks_per_cu"] <= 20 and 0 <= cfg["nee_blocks_per_cu"] <= 20
    assert 0 <= cfg["photon_blocks_per_cu"] <= 64
    assert cfg["photon_order"] in (0, 1)
    assert T.launch_config() == cfg
    assert T.stats()["iterations"] == 0  # reset after tuning
    F = neb.BatchRenderer(scenes, flags=neb.FLAG_SINGLE_THREAD_OCTREE, spp=spp)
    assert cfg["concurrent"] in (0, 1)
    # the other photon order, every launch on one stream
    F.set_launch_config(64, 4, 8, 1 - cfg["photon_order"], concurrent=0)
    T.render(3)
    F.render(3)
    for s in range(len(scenes)):
        nt, it_ = T.octree(s)
        nf, if_ = F.octree(s)
        assert np.array_equal(nt, nf), s
        assert close(T.image_host(s), F.image_host(s), rtol=1e-3), s
    with pytest.raises(neb.NebError):
        F.set_launch_config(40, 4, 8)
    T.close()
    F.close()
