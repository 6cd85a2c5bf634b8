"""FP64 reference of the learned density inside a render (plain numpy).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and nothing else.  The
product library shares no code with it.

The paper converts NEE irradiance into photon flux with the density of NEE
vertices, Phi = dE / rho (eq. flux), and estimates rho with its octree
(Sec. 5.3, eq. octdensity; the five-probe query of Appendix B,
get_density_robust).  A learned model may stand in for that query; the
octree stays the judge and the fallback.  This module states that use of
the model step by step, for the oracle's density hook:

1. training iterations 1..T: the robust octree gives rho, and its NEE
   vertices with rho > 0 form the training pool (position, normal, log rho);
2. later iterations: the octree is frozen (the oracle's ``freeze_after``),
   the model gives rho_model = exp(mu + sigma * y(encode(q, n))), q being
   the position normalised to the octree's box;
3. probes: in the first model iteration every vertex, then every
   ``probe_every`` iterations each vertex whose own uniform u (24 bits,
   counter (pixel, iteration, depth, PROBE), key (model seed, 'PROB'))
   satisfies u * n < probes * 2^24, n the iteration's vertex count.  A
   probe is over the bound when |rho_model - rho_octree| > bound *
   rho_octree, or rho_octree = 0 < rho_model;
4. gate: the octree box is cut into 32^3 regions; a region keeps the model
   while the model's densities summed over its probes so far lie within the
   bound of the octree's densities summed over the same probes (none probed:
   it keeps it); elsewhere rho is the robust octree's.  Probe by probe the
   octree's counting noise exceeds a 10 % bound, so the gate judges the
   model's bias over the region, where that noise averages out.

Region indices are taken in FP32 like the octree's cell addressing
(integers decided by floating point are decided in one precision on both
sides).  The model itself is evaluated by ``oracle.mlp`` (with bf16=True,
the operand rounding of the matrix cores).
"""
import numpy as np

from . import mlp as M
from . import oracle as O

REGION_RES = 32
TAG_PROBE = 6
PROBE_KEY1 = 0x50524F42  # 'PROB'


def region_index(pos, min_bound, size_inv):
    """Region x + 32 (y + 32 z) of each position (FP32 addressing)."""
    p = np.asarray(pos, np.float32)
    q = (p - min_bound.astype(np.float32)) * size_inv.astype(np.float32)
    r = np.clip((q * np.float32(REGION_RES)).astype(np.int64), 0, REGION_RES - 1)
    return r[:, 0] + REGION_RES * (r[:, 1] + REGION_RES * r[:, 2])


def normalised(pos, min_bound, size_inv):
    q = (np.asarray(pos, np.float64) - min_bound.astype(np.float64)) * size_inv.astype(np.float64)
    return np.clip(q, 0.0, 1.0 - 2.0 ** -24)


def probe_mask(pixel, depth, it, n, probes, seed):
    """The vertices a random probe round picks (each by its own draw)."""
    out = np.zeros(len(pixel), bool)
    lim = int(probes) << 24
    for i, (px, d) in enumerate(zip(pixel, depth)):
        u = int(O.philox([int(px), int(it), int(d), TAG_PROBE], [int(seed) & 0xFFFFFFFF, PROBE_KEY1])[0]) >> 8
        out[i] = u * int(n) < lim
    return out


class LearnedDensity:
    """Density hook of an oracle render with the learned density.

    theta, mu, sigma: the model (flat parameters, log rho = mu + sigma y).
    octree: the oracle octree of the render (its box normalises positions).
    """

    def __init__(self, theta, mu, sigma, octree, train_iterations, probe_every=8, probes=4096,
                 max_rel_error=0.1, seed=1, bf16=True, collect=False):
        self.theta = np.asarray(theta, np.float64)
        self.mu, self.sigma = float(mu), float(sigma)
        self.T = int(train_iterations)
        self.probe_every, self.probes = int(probe_every), int(probes)
        self.max_rel = float(max_rel_error)
        self.seed = int(seed)
        self.bf16 = bf16
        self.min_bound, self.size_inv = octree.box()
        n = REGION_RES ** 3
        self.total = np.zeros(n, np.int64)
        self.bad = np.zeros(n, np.int64)
        self.sum_model = np.zeros(n)
        self.sum_octree = np.zeros(n)
        self.gate = np.ones(n, bool)
        self.collect = collect
        self.pool = []          # training iterations: (pos, nrm, log rho) of rho > 0
        self.served = 0         # model-served densities
        self.fallback = 0       # octree-served densities in model iterations
        self.n_probes = 0
        self.n_bad = 0

    def model_rho(self, pos, nrm):
        q = normalised(pos, self.min_bound, self.size_inv)
        y, _ = M.forward(self.theta, M.encode(q, np.asarray(nrm, np.float64)), bf16=self.bf16)
        return np.exp(self.mu + self.sigma * y)

    def __call__(self, pos, nrm, pixel, depth, it, rho):
        if it <= self.T:
            if self.collect:
                ok = rho > 0
                self.pool.append((pos[ok], nrm[ok], np.log(rho[ok])))
            return rho
        j = it - self.T
        ro = rho
        rm = self.model_rho(pos, nrm)
        reg = region_index(pos, self.min_bound, self.size_inv)
        if j == 1 or (j - 1) % self.probe_every == 0:
            probed = np.ones(len(rho), bool) if j == 1 else probe_mask(pixel, depth, it, len(rho), self.probes,
                                                                     self.seed)
            over = np.where(ro > 0, np.abs(rm - ro) > self.max_rel * ro, rm > 0)
            np.add.at(self.total, reg[probed], 1)
            np.add.at(self.bad, reg[probed & over], 1)
            np.add.at(self.sum_model, reg[probed], rm[probed])
            np.add.at(self.sum_octree, reg[probed], ro[probed])
            self.n_probes += int(probed.sum())
            self.n_bad += int((probed & over).sum())
            so, sm = self.sum_octree, self.sum_model
            within = np.where(so > 0, np.abs(sm - so) <= self.max_rel * so, ~(sm > 0))
            self.gate = (self.total == 0) | within
        keep = self.gate[reg]
        self.served += int(keep.sum())
        self.fallback += int((~keep).sum())
        return np.where(keep, rm, ro)

    def pool_arrays(self):
        pos = np.concatenate([p for p, _, _ in self.pool])
        nrm = np.concatenate([n for _, n, _ in self.pool])
        t = np.concatenate([t for _, _, t in self.pool])
        return pos, nrm, t


def train(pos, nrm, log_rho, min_bound, size_inv, steps, batch, seed, lr=2e-3):
    """Fits a model to (pos, nrm, log rho) with Adam in FP64: mu, sigma from
    the targets, then `steps` steps on batches drawn with numpy's generator.
    Returns (theta, mu, sigma, final loss on the whole set)."""
    q = normalised(pos, min_bound, size_inv)
    x = M.encode(q, np.asarray(nrm, np.float64))
    t = np.asarray(log_rho, np.float64)
    mu, sigma = float(t.mean()), float(max(t.std(), 1e-3))
    tn = (t - mu) / sigma
    theta = M.init_params(seed)
    opt = M.Adam(M.N_PARAMS, lr=lr)
    rng = np.random.default_rng(seed)
    for _ in range(steps):
        idx = rng.integers(0, len(t), batch)
        _, g = M.loss_and_grad(theta, x[idx], tn[idx])
        theta = opt.step(theta, g)
    loss, _ = M.loss_and_grad(theta, x, tn)
    return theta, mu, sigma, loss
