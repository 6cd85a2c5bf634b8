"""Pins of the oracle's learned-density reference (oracle/learned.py): the
model in place of the octree query (Sec. 5.3, eq. octdensity; Appendix B
get_density_robust), probe-gated per region with the octree as fallback.

- A model whose output is a constant c, with a bound no probe exceeds,
  renders the model iterations exactly as the oracle's analytic density
  rho = c does (the hook only replaces rho).
- A bound every probe exceeds, with every vertex probed, sends every
  vertex back to the octree: the model iterations render exactly as the
  robust octree frozen after T.
- Freezing: the octree takes no deposits after T (ledger and deposits
  stop).
- Random probes: each vertex is picked by its own draw, so the choice does
  not depend on the order of the vertices, and the expected count is the
  requested one.
- Training: the FP64 fit reaches a small loss on a smooth target.
"""
import numpy as np
import pytest

from neb_inputs import tiny_box
from oracle import learned as LD
from oracle import mlp as M

T = 2
N_MODEL = 2


def _constant_model(c):
    theta = np.zeros(M.N_PARAMS)
    return theta, float(np.log(c)), 1.0


def _split_render(oracle, sc, hook, octree):
    a = oracle.render(sc, n_iter=T, octree=octree, freeze_after=T, density_hook=hook)
    b = oracle.render(sc, n_iter=N_MODEL, first_iter=T + 1, octree=octree, freeze_after=T, density_hook=hook)
    return a, b


def test_constant_model_equals_constant_density(oracle):
    sc = tiny_box(width=24, height=24)
    lo, hi = oracle.OracleScene(sc).bounds()
    oc = oracle.Octree(lo, hi, sc.octree_capacity)
    c = 2500.0
    theta, mu, sigma = _constant_model(c)
    hook = LD.LearnedDensity(theta, mu, sigma, oc, T, probe_every=1, probes=100, max_rel_error=1e30)
    _, b = _split_render(oracle, sc, hook, oc)
    ref = oracle.render(sc, n_iter=N_MODEL, first_iter=T + 1, density_mode=oracle.DENSITY_ANALYTIC, rho0=c,
                        cam_weight=0.0)
    assert hook.fallback == 0 and hook.served == b["stats"]["vertices"]
    assert b["stats"]["photons"] == ref["stats"]["photons"] > 0
    for t in ("e", "E", "P"):
        assert np.allclose(b["tech"][t], ref["tech"][t], rtol=1e-12, atol=1e-300), t


def test_zero_bound_falls_back_to_frozen_octree(oracle):
    sc = tiny_box(width=24, height=24)
    lo, hi = oracle.OracleScene(sc).bounds()
    oc1 = oracle.Octree(lo, hi, sc.octree_capacity)
    theta, mu, sigma = _constant_model(2500.0)
    # every vertex is probed in every model iteration (probes >= vertices)
    hook = LD.LearnedDensity(theta, mu, sigma, oc1, T, probe_every=1, probes=10 ** 7, max_rel_error=1e-12)
    a, b = _split_render(oracle, sc, hook, oc1)
    oc2 = oracle.Octree(lo, hi, sc.octree_capacity)
    ra = oracle.render(sc, n_iter=T, octree=oc2, freeze_after=T)
    rb = oracle.render(sc, n_iter=N_MODEL, first_iter=T + 1, octree=oc2, freeze_after=T)
    assert hook.served == 0 and hook.fallback == b["stats"]["vertices"]
    assert not hook.gate[hook.total > 0].any() and (hook.total > 0).any()
    # (equal up to the order of the oracle's per-thread sums)
    for t in ("e", "E", "P"):
        assert np.allclose(a["tech"][t], ra["tech"][t], rtol=1e-10, atol=0), t
        assert np.allclose(b["tech"][t], rb["tech"][t], rtol=1e-10, atol=0), t
    # frozen after T: the model iterations deposit nothing
    _, ia = oc1.export()
    assert ia["deposits"] == a["stats"]["vertices"] == ia["ledger"]


def test_probe_choice_is_per_vertex_and_has_the_requested_rate():
    rng = np.random.default_rng(3)
    n = 4000
    pixel = rng.integers(0, 1 << 20, n)
    depth = rng.integers(1, 8, n)
    m = LD.probe_mask(pixel, depth, 9, n, 1000, seed=5)
    perm = rng.permutation(n)
    m2 = LD.probe_mask(pixel[perm], depth[perm], 9, n, 1000, seed=5)
    assert np.array_equal(m[perm], m2)
    # binomial(n, 1/4): mean 1000, sd ~27
    assert abs(int(m.sum()) - 1000) < 5 * 27
    # another iteration draws another subset
    m3 = LD.probe_mask(pixel, depth, 10, n, 1000, seed=5)
    assert 0.15 < np.mean(m & m3) / np.mean(m) < 0.35


def test_region_index_follows_the_box():
    lo = np.float32([0.0, 0.0, 0.0])
    inv = np.float32([0.5, 0.25, 1.0])      # box 2 x 4 x 1
    p = np.float32([[0.0, 0.0, 0.0], [1.99, 3.99, 0.99], [1.0, 2.0, 0.5], [-1.0, 9.0, 0.2]])
    r = LD.region_index(p, lo, inv)
    assert list(r) == [0, 31 + 32 * (31 + 32 * 31), 16 + 32 * (16 + 32 * 16), 0 + 32 * (31 + 32 * 6)]


def test_training_fits_a_smooth_log_density():
    rng = np.random.default_rng(2)
    pos = rng.uniform(0, 1, (2000, 3))
    nrm = rng.normal(size=(2000, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    t = 3.0 + np.sin(3 * pos[:, 0]) + 0.5 * pos[:, 1]
    theta, mu, sigma, loss = LD.train(pos, nrm, t, np.zeros(3, np.float32), np.ones(3, np.float32), steps=300,
                                      batch=512, seed=1)
    assert loss < 0.02, loss
    q = LD.normalised(pos, np.zeros(3, np.float32), np.ones(3, np.float32))
    y, _ = M.forward(theta, M.encode(q, nrm))
    assert np.sqrt(np.mean((mu + sigma * y - t) ** 2)) < 0.15
    assert mu == pytest.approx(t.mean())
