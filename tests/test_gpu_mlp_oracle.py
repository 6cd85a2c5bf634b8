"""The learned density in a render, GPU against the FP64 oracle.

The model stands in for the octree's density query (Sec. 5.3, eq.
octdensity; Appendix B get_density_robust), judged by the octree and
falling back to it per region (oracle/learned.py states the rules).  The
model compared here is trained by the oracle: T iterations of the robust
octree give the training pool (the oracle's own densities), and an FP64
Adam fit on it gives the weights; both sides then render with those
weights and no further training, from the same seed:

- the octree of the training iterations: the deterministic single-thread
  GPU tree against the oracle's sequential tree;
- model iterations: probes chosen by each vertex's own draw, the 32^3
  region gates (the model's densities summed over a region's probes within
  the bound of the octree's), the octree fallback elsewhere; the gates
  agree region by region, and so do the probe counts;
- the images of the model iterations (the sums after T + N iterations
  minus those after T) agree with the oracle's element by element,
  technique by technique (relative RMSE, R22).
"""
import numpy as np
import pytest

from neb_inputs import tiny_box
from oracle import learned as LD
from parity import technique_errors

pytestmark = pytest.mark.gpu

T = 2
N_MODEL = 6
PROBE_EVERY = 2
PROBES = 2000
BOUND = 0.1
SEED = 5


@pytest.fixture(scope="module")
def neb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_00573_amd import neb as N
    N.lib()
    return N


def _oracle_model_run(oracle, sc):
    """The oracle's training iterations, the model fitted to their pool,
    and the oracle's model iterations."""
    osc = oracle.OracleScene(sc)
    lo, hi = osc.bounds()
    oc = oracle.Octree(lo, hi, sc.octree_capacity)
    collector = LD.LearnedDensity(np.zeros(LD.M.N_PARAMS), 0.0, 1.0, oc, T, collect=True)
    a = oracle.render(sc, n_iter=T, octree=oc, oscene=osc, freeze_after=T, density_hook=collector)
    pos, nrm, t = collector.pool_arrays()
    mb, inv = oc.box()
    theta, mu, sigma, loss = LD.train(pos, nrm, t, mb, inv, steps=300, batch=2048, seed=SEED)
    hook = LD.LearnedDensity(theta, mu, sigma, oc, T, probe_every=PROBE_EVERY, probes=PROBES, max_rel_error=BOUND,
                             seed=SEED)
    b = oracle.render(sc, n_iter=N_MODEL, first_iter=T + 1, octree=oc, oscene=osc, freeze_after=T,
                      density_hook=hook)
    return a, b, hook, (theta, mu, sigma, loss)


def _gpu_model_run(neb, sc, model):
    theta, mu, sigma, _ = model
    R = neb.Renderer(sc, density_mode=neb.DENSITY_MLP, flags=neb.FLAG_SINGLE_THREAD_OCTREE)
    R.configure_mlp(train_iterations=T, steps_per_iteration=0, probe_every=PROBE_EVERY, probes=PROBES,
                    max_rel_error=BOUND, seed=SEED)
    R.set_mlp_model(theta.astype(np.float32), mu, sigma)
    R.render(T)
    first = {k: v.astype(np.float64) * T for k, v in R.technique_images_host().items()}
    st_t = R.stats()
    R.render(N_MODEL)
    tech = {k: v.astype(np.float64) * (T + N_MODEL) - first[k] for k, v in R.technique_images_host().items()}
    out = dict(tech=tech, stats=R.stats(), stats_t=st_t, status=R.mlp_status(), gates=R.mlp_gates(),
               octree=R.octree())
    R.close()
    return out


def test_learned_density_render_matches_oracle(neb, oracle):
    sc = tiny_box()
    a, b, hook, model = _oracle_model_run(oracle, sc)
    g = _gpu_model_run(neb, sc, model)
    print(f"\nmodel: loss {model[3]:.3f}, mu {model[1]:.3f}, sigma {model[2]:.3f}", flush=True)
    # the training iterations built the same tree
    nodes_g, info_g = g["octree"]
    nodes_o, info_o = a["octree"].export()
    assert info_g["deposits"] == g["stats_t"]["vertices"] == info_o["deposits"]
    assert np.mean(nodes_g == nodes_o) > 0.99
    # frozen after T on both sides
    assert g["stats"]["oct_deposits"] == g["stats_t"]["oct_deposits"]
    # probes and gates
    s = g["status"]
    gate_g = g["gates"]["gate"].ravel().astype(bool)
    tot_g = g["gates"]["probes"].ravel()
    both = (tot_g > 0) & (hook.total > 0)
    agree = float(np.mean(gate_g[both] == hook.gate[both]))
    print(f"probes {s['probes']}/{hook.n_probes} over the bound {s['probes_bad']}/{hook.n_bad}; regions probed "
          f"{int((tot_g > 0).sum())}/{int((hook.total > 0).sum())}, disabled {s['regions_disabled']}/"
          f"{int((~hook.gate).sum())}, gates equal {agree:.4f}; fallback {s['fallback_queries']}/{hook.fallback}; "
          f"served probes over the bound {s['probes_served_bad']}/{s['probes_served']}", flush=True)
    assert s["probes"] == pytest.approx(hook.n_probes, rel=2e-3)
    assert s["probes_bad"] == pytest.approx(hook.n_bad, rel=0.02, abs=5)
    assert both.sum() > 50 and agree >= 0.99
    assert 0 < s["regions_disabled"] < int((tot_g > 0).sum())
    assert s["fallback_queries"] == pytest.approx(hook.fallback, rel=0.02, abs=10)
    assert s["probes_served"] > 0
    # images of the model iterations
    terr = technique_errors(g["tech"], b["tech"], 1)
    print(f"model iterations: technique errors {terr}", flush=True)
    assert b["tech"]["P"].sum() > 0.01 * sum(b["tech"][t].sum() for t in ("e", "E", "P"))
    for t, v in terr.items():
        assert v < 0.01, (t, v)
    for k in ("vertices", "photons", "merges"):
        assert g["stats"][k] - g["stats_t"][k] == pytest.approx(b["stats"][k], rel=2e-3), k
