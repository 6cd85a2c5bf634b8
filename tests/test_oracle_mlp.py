"""Pins of the FP64 learned-density reference (oracle/mlp.py).

- bfloat16 rounding against hand-placed halfway cases (ties to even);
- the encoding against closed-form sines and cosines at chosen points;
- the forward pass against a hand-built network with a closed-form output
  (pins the orientation of W, the biases and the ReLUs);
- the analytic gradient against central finite differences;
- Adam against its closed form for a constant gradient;
- a 256-sample set is fitted to a loss below 1e-4.
"""
import numpy as np
import pytest

from oracle import mlp as M


def test_bf16_rounding_halfway_cases():
    one = 1.0
    u = 2.0 ** -7  # bfloat16 spacing at 1
    vals = np.array([one, one + u / 2, one + 3 * u / 2, one + u / 2 + 2.0 ** -20, -(one + 3 * u / 2), 0.0])
    want = np.array([one, one, one + 2 * u, one + u, -(one + 2 * u), 0.0])
    assert np.array_equal(M.bf16_round(vals), want)
    # exactly representable values survive
    x = np.array([0.5, -2.0, 1.5, 3.0 + 2.0 ** -6 * 2])
    assert np.array_equal(M.bf16_round(x), x)


def test_encoding_closed_form():
    q = np.array([[0.25, 0.5, 0.75]])
    n = np.array([[0.0, 0.0, 1.0]])
    x = M.encode(q, n)[0]
    assert x.shape == (80,)
    assert np.array_equal(x[:6], [0.25, 0.5, 0.75, 0.0, 0.0, 1.0])
    s2 = np.sqrt(0.5)
    # q0 = 1/4: sin/cos of pi/4, pi/2, pi, 2 pi, 4 pi, 8 pi
    want_q0 = [s2, s2, 1, 0, 0, -1, 0, 1, 0, 1, 0, 1]
    assert np.allclose(x[6:18], want_q0, atol=1e-12)
    # q1 = 1/2: pi/2, pi, 2 pi, ...
    want_q1 = [1, 0, 0, -1, 0, 1, 0, 1, 0, 1, 0, 1]
    assert np.allclose(x[18:30], want_q1, atol=1e-12)
    # n2 = 1: sin(2^f pi) = 0, cos(pi) = -1 then +1
    want_n2 = [0, -1, 0, 1, 0, 1, 0, 1, 0, 1, 0, 1]
    assert np.allclose(x[66:78], want_n2, atol=1e-12)
    # n0 = 0: sin 0 = 0, cos 0 = 1
    assert np.allclose(x[42:54], [0, 1] * 6, atol=0)
    assert x[78] == 0 and x[79] == 0


def test_forward_hand_built_network():
    theta = np.zeros(M.N_PARAMS)
    p = M.unflatten(theta)
    p["W1"][0, 0] = 1.0      # unit 0 of layer 1 reads feature 0 (q0)
    p["b1"][0] = 0.5
    p["W1"][0, 1] = 1.0      # unit 1: q0 - 2 < 0, cut by the ReLU
    p["b1"][1] = -2.0
    p["W2"][0, 0] = 2.0
    p["W2"][1, 0] = 100.0    # would show if unit 1 leaked through
    p["W3"][0, 3] = 1.0
    p["W2"][0, 5] = -1.0     # unit 5 of layer 2 is negative, cut by its ReLU
    p["W3"][5, 3] = 100.0
    p["b3"][3] = -0.25
    p["w4"][3] = 3.0
    p["b4"][0] = 1.0
    q = np.array([[0.1, 0.9, 0.3], [0.7, 0.2, 0.4]])
    n = np.array([[0, 1.0, 0], [1.0, 0, 0]])
    y, _ = M.forward(theta, M.encode(q, n))
    want = 3.0 * (2.0 * (q[:, 0] + 0.5) - 0.25) + 1.0
    assert np.allclose(y, want, rtol=1e-14)
    # a negative pre-activation at the last hidden layer gives y = b4
    p["b3"][3] = -10.0
    y, _ = M.forward(theta, M.encode(q, n))
    assert np.array_equal(y, [1.0, 1.0])


def _batch(seed, N):
    rng = np.random.default_rng(seed)
    q = rng.uniform(0, 1, (N, 3))
    n = rng.normal(size=(N, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    t = np.sin(3 * q[:, 0]) + 0.5 * np.cos(2 * q[:, 1]) + n[:, 2]
    return M.encode(q, n), t


def test_gradient_matches_central_differences():
    x, t = _batch(1, 7)
    theta = M.init_params(3)
    theta[M.N_PARAMS - 1] = 0.3
    _, g = M.loss_and_grad(theta, x, t)
    rng = np.random.default_rng(5)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SHAPES])
    idx = set(rng.choice(M.N_PARAMS, 300, replace=False).tolist())
    for a, b in zip(offs[:-1], offs[1:]):   # a few entries of every tensor, ends included
        idx |= {int(a), int(b) - 1, int((a + b) // 2)}
    h = 1e-6
    for i in sorted(idx):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.loss_and_grad(tp, x, t)[0] - M.loss_and_grad(tm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
    # padded inputs carry no gradient
    W1g = M.unflatten(g)["W1"]
    assert np.all(W1g[78:] == 0)


def test_bf16_gradient_close_to_exact():
    x, t = _batch(2, 512)
    theta = M.init_params(4)
    _, g = M.loss_and_grad(theta, x, t)
    _, gb = M.loss_and_grad(theta, x, t, bf16=True)
    for name, _ in M.SHAPES:
        a, b = M.unflatten(g)[name].ravel(), M.unflatten(gb)[name].ravel()
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
        assert cos > 0.99, name


def test_adam_closed_form_for_constant_gradient():
    rng = np.random.default_rng(9)
    theta0 = rng.normal(size=50)
    g = rng.normal(size=50)
    opt = M.Adam(50, lr=1e-2)
    th = theta0.copy()
    for step in range(1, 6):
        th = opt.step(th, g)
        # both moments are bias-corrected to g and g^2 exactly
        want = theta0 - step * 1e-2 * g / (np.abs(g) + 1e-8)
        assert np.allclose(th, want, rtol=0, atol=1e-12)


@pytest.mark.slow
def test_overfits_256_samples():
    x, t = _batch(7, 256)
    theta = M.init_params(11)
    opt = M.Adam(M.N_PARAMS, lr=2e-3)
    loss = None
    for step in range(4000):
        loss, g = M.loss_and_grad(theta, x, t)
        theta = opt.step(theta, g)
        if loss < 1e-4:
            break
    assert loss < 1e-4, loss
