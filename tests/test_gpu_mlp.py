"""The learned density's matrix-core kernels against the FP64 reference.

The reference (oracle/mlp.py) is run with the same bf16 operand rounding
the kernels apply (encoded inputs, hidden activations and deltas feeding
the matrix cores, weights W1..W3), so the remaining differences are FP32
versus FP64 accumulation, FP32 sine/cosine, and the rare bf16 rounding
that these flip at a tie.  Bounds:
- outputs: median |dy| <= 1e-5, 99th percentile <= 2e-3, max <= 5e-2;
- gradients, per tensor: cosine >= 0.999 and relative L2 <= 1e-2;
- an Adam step moves the parameters as the reference step does.
Batches of 1000 samples span many 16-sample tiles and a ragged last tile.
"""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def neb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_00573_amd import neb as N
    N.lib()
    return N


def _inputs(seed, n):
    rng = np.random.default_rng(seed)
    q = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    nn = rng.normal(size=(n, 3))
    nn = (nn / np.linalg.norm(nn, axis=1, keepdims=True)).astype(np.float32)
    t = (np.sin(3 * q[:, 0]) + 0.5 * np.cos(2 * q[:, 1]) + nn[:, 2]).astype(np.float32)
    return q, nn, t


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _theta(seed):
    th = M.init_params(seed).astype(np.float32)
    rng = np.random.default_rng(seed + 100)
    th[M.N_PARAMS - 65:] += rng.normal(0, 0.1, 65).astype(np.float32)  # nonzero b3/w4/b4 tail
    return th


@pytest.mark.parametrize("n", [1, 16, 1000])
def test_forward_matches_reference(neb, n):
    th = _theta(3)
    q, nn, _ = _inputs(5, n)
    m = neb.Mlp(init=th, max_batch=1024)
    y = m.infer(_dev(q), _dev(nn)).cpu().numpy().astype(np.float64)
    ref, _ = M.forward(th.astype(np.float64), M.encode(q.astype(np.float64), nn.astype(np.float64)), bf16=True)
    d = np.abs(y - ref)
    assert np.median(d) <= 1e-5, np.median(d)
    assert np.percentile(d, 99) <= 2e-3
    assert d.max() <= 5e-2
    # normalisation: log rho = mu + sigma * y
    m.set_normalization(2.0, 0.5)
    y2 = m.infer(_dev(q), _dev(nn)).cpu().numpy().astype(np.float64)
    assert np.allclose(y2, 2.0 + 0.5 * y, rtol=1e-6, atol=1e-6)
    m.close()


def _cos_rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(a @ b / (np.linalg.norm(a) * nb + 1e-300)), float(np.linalg.norm(a - b) / (nb + 1e-300))


def test_gradient_matches_reference(neb):
    th = _theta(7)
    q, nn, t = _inputs(8, 1000)
    m = neb.Mlp(init=th, max_batch=1024)
    g, loss = m.gradient(_dev(q), _dev(nn), _dev(t))
    g = g.cpu().numpy()
    x = M.encode(q.astype(np.float64), nn.astype(np.float64))
    lref, gref = M.loss_and_grad(th.astype(np.float64), x, t.astype(np.float64), bf16=True)
    assert loss == pytest.approx(lref, rel=2e-3)
    G, R = M.unflatten(g.astype(np.float64)), M.unflatten(gref)
    for name, _ in M.SHAPES:
        if name == "W1":   # the two zero-padded input rows carry no gradient
            assert np.all(G[name][78:] == 0)
        cos, rel = _cos_rel(G[name], R[name])
        assert cos >= 0.999 and rel <= 1e-2, (name, cos, rel)
    # the bf16 kernels also track the exact FP64 gradient
    _, gex = M.loss_and_grad(th.astype(np.float64), x, t.astype(np.float64))
    cos, _ = _cos_rel(g, gex)
    assert cos >= 0.99
    # a repeated call gives the same gradient (the accumulator is cleared)
    g2, _ = m.gradient(_dev(q), _dev(nn), _dev(t))
    assert np.allclose(g2.cpu().numpy(), g, rtol=1e-5, atol=1e-9)
    m.close()


def test_adam_step_matches_reference(neb):
    th = _theta(9)
    q, nn, t = _inputs(10, 1000)
    m = neb.Mlp(init=th, max_batch=1024)
    lr = 1e-3
    m.train_step(_dev(q), _dev(nn), _dev(t), lr=lr)
    after = m.params().astype(np.float64)
    x = M.encode(q.astype(np.float64), nn.astype(np.float64))
    _, gref = M.loss_and_grad(th.astype(np.float64), x, t.astype(np.float64), bf16=True)
    opt = M.Adam(M.N_PARAMS, lr=lr)
    want = opt.step(th.astype(np.float64), gref)
    step_gpu, step_ref = after - th, want - th
    # the first step is lr * g / (|g| + eps): compare where the gradient is well resolved
    sure = np.abs(gref) > 1e-3 * np.abs(gref).max()
    assert sure.sum() > 1000
    assert np.allclose(step_gpu[sure], step_ref[sure], rtol=0, atol=0.02 * lr)
    assert np.all(np.abs(step_gpu) <= lr * 1.0001 + 1e-7)
    m.close()


def test_training_fits_a_smooth_density(neb):
    import torch
    q, nn, t = _inputs(11, 8192)
    m = neb.Mlp(seed=3, max_batch=8192)
    Q, N_, T = _dev(q), _dev(nn), _dev(t)
    _, loss0 = m.gradient(Q, N_, T)
    for _ in range(400):
        m.train_step(Q, N_, T, lr=3e-3)
    torch.cuda.synchronize()
    _, loss1 = m.gradient(Q, N_, T)
    assert loss1 < 0.02 * loss0, (loss0, loss1)
    m.close()


def test_render_with_learned_density(neb):
    """Room at 128 x 128: two training iterations on the GPU's own kernels,
    then the model with its probes, gates and octree fallback."""
    from neb_inputs import room
    sc = room(width=128, height=128)
    R = neb.Renderer(sc, density_mode=neb.DENSITY_MLP)
    R.configure_mlp(train_iterations=2, steps_per_iteration=100, batch=16384, probe_every=2, probes=512)
    R.render(2)
    st2 = R.stats()
    s = R.mlp_status()
    assert s["phase"] == 0 and s["adam_steps"] == 200
    assert np.isfinite(s["last_loss"]) and s["last_loss"] < 0.5 and s["sigma"] > 0
    R.render(6)
    st = R.stats()
    s = R.mlp_status()
    assert s["phase"] == 1
    # the octree stopped counting after the training iterations
    assert st["oct_deposits"] == st2["oct_deposits"] and st["oct_ledger"] == st["oct_deposits"]
    # every vertex of the first model iteration was probed, then 512 every 2 iterations
    assert s["probes"] >= st2["vertices"] // 2 and s["regions_probed"] > 0
    assert s["regions_disabled"] < s["regions_probed"]
    tech = R.technique_images_host()
    for t in tech.values():
        assert np.all(np.isfinite(t))
    assert s["probes_served"] > 0 and 0 <= s["probes_served_bad"] <= s["probes_served"]
    # (the rendered images are compared with the oracle's evaluation of the
    # same gated model in tests/test_gpu_mlp_oracle.py)
    # a tiny error bound sends every probed region back to the octree
    R.configure_mlp(train_iterations=2, steps_per_iteration=20, batch=4096, probe_every=2, probes=512,
                    max_rel_error=1e-7)
    R.render(4)
    s = R.mlp_status()
    assert s["regions_disabled"] == s["regions_probed"] > 0
    assert s["fallback_queries"] > 0
    R.close()


def test_room_full_size_model_matches_reference(neb):
    """Room at its full size with the default model settings (4 training
    iterations of 250 Adam steps on 65 536 draws): the trained model's
    log density at sampled surface points equals the FP64 reference's
    evaluation of the same weights (bf16 operand rounding emulated)."""
    import torch
    from neb_inputs import room
    sc = room()
    R = neb.Renderer(sc, density_mode=neb.DENSITY_MLP, flags=neb.FLAG_RECORD_PATHS)
    R.render(5)
    s = R.mlp_status()
    assert s["phase"] == 1 and s["adam_steps"] == 1000
    assert s["last_loss"] < 0.2
    w = R.mlp_weights()
    rec = R.records()
    R.close()
    # sampled first-hit points of the recorded paths, normalised to the octree box
    hits = rec[:, 0][(rec[:, 0]["type"] >= 1) & (rec[:, 0]["type"] <= 4)]
    rng = np.random.default_rng(1)
    pos = hits["pos"][rng.choice(len(hits), 2000, replace=False)].astype(np.float64)
    lo, hi = sc.bbox()
    size = (hi.astype(np.float64) - lo) * 1.002
    q = np.clip((pos - (lo - size * (0.001 / 1.002))) / size, 0, 1 - 1e-7).astype(np.float32)
    nn = rng.normal(size=(len(q), 3))
    nn = (nn / np.linalg.norm(nn, axis=1, keepdims=True)).astype(np.float32)
    m = neb.Mlp(init=w, max_batch=2048)
    m.set_normalization(s["mu"], s["sigma"])
    got = m.infer(_dev(q), _dev(nn)).cpu().numpy().astype(np.float64)
    y, _ = M.forward(w.astype(np.float64), M.encode(q.astype(np.float64), nn.astype(np.float64)), bf16=True)
    want = s["mu"] + s["sigma"] * y
    d = np.abs(got - want)
    assert np.median(d) <= 1e-4 and np.percentile(d, 99) <= 5e-3 and d.max() <= 5e-2, (np.median(d), d.max())
    m.close()
    torch.cuda.synchronize()
