"""FP64 reference of the learned density model (plain numpy).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and nothing else.  The
product library shares no code with it.

The model stands in for the octree's density query (Sec. 5, eq.
octdensity): a multilayer perceptron maps a surface point and its normal to
the logarithm of the density of NEE vertices there, and is fitted to the
octree's own robust densities.  The paper has no such model; its shape is
fixed by the design this library follows:

- input encoding (80 features): the point normalised to the octree's
  bounding box, q in [0, 1)^3, the unit normal n, then for each of the six
  coordinates c = (q0, q1, q2, n0, n1, n2) and octave f = 0..5 the pair
  sin(2^f pi c), cos(2^f pi c) (feature 6 + 12 c + 2 f and the next one),
  then two zeros;
- three hidden layers of width 64 with ReLU, z_l = W_l^T h_{l-1} + b_l,
  h_l = max(z_l, 0), and a linear output y = w4 . h3 + b4;
- the output is normalised: log rho = mu + sigma * y;
- loss: mean squared error of y against (log rho_target - mu) / sigma over
  a batch; Adam (Kingma and Ba, ICLR 2015) on FP32 master parameters.

Flat parameter layout (both sides use it): W1 (80 x 64, row k holds the
weights from input feature k), b1 (64), W2 (64 x 64), b2, W3 (64 x 64),
b3, w4 (64), b4 (1): 13569 values.

``bf16=True`` reproduces the points where the GPU kernels round operands to
bfloat16 (round to nearest, ties to even) while every sum stays FP64: the
encoded input and the hidden activations h1, h2 that feed the matrix
cores, the weights W1..W3, and in the backward pass the deltas that feed
the matrix cores.  Biases, w4, b4, h3 and every accumulation stay wide.
"""
import numpy as np

N_IN = 80
N_ENC = 78
WIDTH = 64
OCTAVES = 6
SHAPES = [("W1", (N_IN, WIDTH)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("w4", (WIDTH,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(theta):
    """Views of the named tensors inside the flat vector."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def bf16_round(x):
    """Round to the nearest bfloat16 value (ties to even), returned as
    float64.  Goes through float32 first, as a float32 operand would."""
    a = np.asarray(x, np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) >> 16 << 16
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def encode(q, n):
    """(N, 3) normalised points and (N, 3) normals -> (N, 80) features."""
    q = np.asarray(q, np.float64)
    n = np.asarray(n, np.float64)
    N = q.shape[0]
    x = np.zeros((N, N_IN))
    x[:, 0:3] = q
    x[:, 3:6] = n
    coords = np.concatenate([q, n], axis=1)
    for c in range(6):
        for f in range(OCTAVES):
            a = (2.0 ** f) * np.pi * coords[:, c]
            x[:, 6 + 12 * c + 2 * f] = np.sin(a)
            x[:, 6 + 12 * c + 2 * f + 1] = np.cos(a)
    return x


def init_params(seed):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shp)
        else:
            fan_in = shp[0]
            bound = np.sqrt(6.0 / fan_in)
            p[name] = rng.uniform(-bound, bound, shp)
    return flatten(p)


def forward(theta, x, bf16=False):
    """Output y (N,) and the cache the backward pass needs."""
    p = unflatten(np.asarray(theta, np.float64))
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    x0 = r(x)
    z1 = x0 @ W1 + p["b1"]
    h1 = np.maximum(z1, 0.0)
    h1r = r(h1)
    z2 = h1r @ W2 + p["b2"]
    h2 = np.maximum(z2, 0.0)
    h2r = r(h2)
    z3 = h2r @ W3 + p["b3"]
    h3 = np.maximum(z3, 0.0)
    y = h3 @ p["w4"] + p["b4"][0]
    return y, {"x0": x0, "z1": z1, "h1r": h1r, "z2": z2, "h2r": h2r, "z3": z3, "h3": h3,
               "W2": W2, "W3": W3}


def loss_and_grad(theta, x, t, bf16=False):
    """Mean squared error over the batch and its gradient (flat), by
    backpropagation through the layers above."""
    p = unflatten(np.asarray(theta, np.float64))
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    y, c = forward(theta, x, bf16)
    N = y.shape[0]
    e = y - np.asarray(t, np.float64)
    loss = float(np.mean(e * e))
    dy = 2.0 * e / N
    g = {"w4": c["h3"].T @ dy, "b4": np.array([dy.sum()])}
    d3 = dy[:, None] * p["w4"][None, :] * (c["z3"] > 0)
    g["b3"] = d3.sum(axis=0)
    d3r = r(d3)
    g["W3"] = c["h2r"].T @ d3r
    d2 = (d3r @ c["W3"].T) * (c["z2"] > 0)
    g["b2"] = d2.sum(axis=0)
    d2r = r(d2)
    g["W2"] = c["h1r"].T @ d2r
    d1 = (d2r @ c["W2"].T) * (c["z1"] > 0)
    g["b1"] = d1.sum(axis=0)
    d1r = r(d1)
    g["W1"] = c["x0"].T @ d1r
    return loss, flatten(g)


class Adam:
    """Adam with bias-corrected moments."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def predict_log_rho(theta, q, n, mu=0.0, sigma=1.0, bf16=False):
    y, _ = forward(theta, encode(q, n), bf16)
    return mu + sigma * y
