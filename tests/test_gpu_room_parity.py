"""GPU against the FP64 oracle where the method does its work: the room
workload's full geometry (a refractive IOR-1.5 sphere of 20 480 facets on a
table, four small emissive spheres, grey walls), path length 8 and its
merge radius, NEB photons on, at reduced image sizes so that the
brute-force oracle finishes in seconds.

Same Philox streams on both sides, so view paths, light samples and
photon walks coincide up to floating-point divergence.

- 64 iterations (the room's reference sample count) at 32 x 32, with
  conventional light photons: the image and every technique image -- e
  (random emitter hits, Sec. 3.3), E (NEE, Sec. 3.1), P (NEB photons, many
  of them refracted through the glass: the caustic paths of Sec. 3.2,
  merged with eq. photonpdf) and LP (eq. stdphotonpdf) -- agree element by
  element within 1 % relative RMSE (R22), with the analytic density (the
  same rho on both sides) and with the single-thread octree (the oracle's
  sequential insertion order).  Path length 8 exercises the whole MIS sum
  of eq. misw.  (A photon walk that meets a glass facet edge within float
  rounding can leave the other side's walk; a single such caustic photon
  moves P by a few per cent of one iteration, so the comparison is made at
  the reference sample count, where they average out.)
- 2 iterations at 96 x 96: every one of the 9216 view paths event by
  event, the work counts (NEE vertices, visible NEE samples, photons,
  photon segments, merges), the NEE and emitter-hit images element by
  element, and the octree's cells.
"""
import numpy as np
import pytest

from neb_inputs import room
from parity import rel_rmse, technique_errors, path_agreement, scene_diag, cell_agreement

pytestmark = pytest.mark.gpu

# analytic density for the room: depth-1 vertices take the camera's
# primary-hit density, deeper ones a constant of the octree's order
# (about 55 k deeper vertices per iteration over ~320 m^2 at 96 x 96)
ROOM_RHO0 = 200.0
TOL = 0.01


@pytest.fixture(scope="module")
def neb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_00573_amd import neb as N
    N.lib()
    return N


def _gpu(neb, sc, mode, n_iter, light_photons=0, flags=0):
    if mode == "analytic":
        g = neb.Renderer(sc, density_mode=neb.DENSITY_ANALYTIC, rho0=ROOM_RHO0, cam_weight=1.0, flags=flags,
                         light_photons=light_photons)
    else:
        g = neb.Renderer(sc, flags=flags | neb.FLAG_SINGLE_THREAD_OCTREE, light_photons=light_photons)
    g.render(n_iter)
    out = dict(img=g.image_host().astype(np.float64), tech=g.technique_images_host(), stats=g.stats())
    if mode == "octree":
        out["octree"] = g.octree()
    g.close()
    return out


def _oracle(oracle, sc, osc, mode, n_iter, light_photons=0):
    if mode == "analytic":
        return oracle.render(sc, n_iter=n_iter, density_mode=oracle.DENSITY_ANALYTIC, rho0=ROOM_RHO0,
                             cam_weight=1.0, oscene=osc, light_photons=light_photons)
    return oracle.render(sc, n_iter=n_iter, oscene=osc, light_photons=light_photons)


def _counts(st, so, lp):
    print(f"vertices {st['vertices']}/{so['vertices']:.0f} nee_visible {st['nee_visible']}/{so['nee_visible']:.0f} "
          f"photons {st['photons']}/{so['photons']:.0f} segments {st['photon_segments']}/{so['photon_segments']:.0f} "
          f"merges {st['merges']}/{so['merges']:.0f} events {st['events']}/{so['events']:.0f}", flush=True)
    assert st["vertices"] == pytest.approx(so["vertices"], rel=1e-3)
    assert st["nee_visible"] == pytest.approx(so["nee_visible"], rel=1e-3)
    assert st["photons"] == pytest.approx(so["photons"], rel=1e-3)
    assert st["photon_segments"] == pytest.approx(so["photon_segments"], rel=1e-3)
    assert st["merges"] == pytest.approx(so["merges"], rel=2e-3)
    if lp:
        assert st["light_photons"] == so["light_photons"]


def _octree(g, o):
    nodes_g, info_g = g["octree"]
    nodes_o, info_o = o["octree"].export()
    agree = cell_agreement(nodes_g, nodes_o)
    print(f"octree: allocated {info_g['allocated']}/{info_o['allocated']}, deposits {info_g['deposits']}/"
          f"{info_o['deposits']}, leaf cells equal {agree:.5f}", flush=True)
    assert info_g["ledger"] == info_g["deposits"]
    assert info_o["ledger"] == info_o["deposits"]
    assert info_g["deposits"] == pytest.approx(info_o["deposits"], rel=1e-3)
    assert info_g["allocated"] == pytest.approx(info_o["allocated"], rel=1e-3)
    assert agree > 0.99


@pytest.mark.parametrize("mode", ["analytic", "octree", "pt_lp"])
def test_room_64_iterations_match_oracle(neb, oracle, mode):
    """pt_lp is path tracing with NEE and light photons, no NEB photons:
    the estimator of the bench's error reference (no density enters it)."""
    sc = room(width=32, height=32)
    n_iter, nlp = 64, 32 * 32
    if mode == "pt_lp":
        g = _gpu(neb, sc, "analytic", n_iter, light_photons=nlp, flags=neb.FLAG_NO_PHOTONS)
        o = oracle.render(sc, n_iter=n_iter, enable_photons=False, light_photons=nlp)
    else:
        g = _gpu(neb, sc, mode, n_iter, light_photons=nlp)
        o = _oracle(oracle, sc, oracle.OracleScene(sc), mode, n_iter, light_photons=nlp)
    err = rel_rmse(g["img"], o["mean"])
    terr = technique_errors(g["tech"], o["tech"], n_iter)
    print(f"\nroom 32x32, 64 iterations, {mode}: image {err:.2e}, techniques {terr}", flush=True)
    _counts(g["stats"], o["stats"], lp=True)
    if mode == "octree":
        _octree(g, o)
    tot = o["sum"].sum()
    # the workload is exercised: every technique carries light
    for t in ("e", "E", "P", "LP"):
        if mode == "pt_lp" and t == "P":
            assert o["tech"][t].sum() == 0 and np.abs(g["tech"][t]).sum() == 0
            continue
        assert o["tech"][t].sum() > 1e-3 * tot, t
    assert err < TOL, err
    for t, v in terr.items():
        assert v < TOL, (t, v)


@pytest.fixture(scope="module")
def room96():
    return room(width=96, height=96)


@pytest.mark.parametrize("mode", ["analytic", "octree"])
def test_room_96_paths_counts_and_nee(neb, oracle, room96, mode):
    """Counts and the NEE / emitter-hit images after 2 iterations; with the
    single-thread octree also the density at every NEE vertex of the last
    iteration: the GPU's robust query on its tree (neb_query_density) at
    the oracle's vertices against the oracle's query on its tree.  (Without
    light photons the P image of 2 iterations is dominated by a few bright
    photons: the vertices whose densities differ by a deposit landing in a
    neighbouring cell move it by tens of per cent; P is compared at 64
    iterations with light photons above.)"""
    import torch
    sc = room96
    n_iter = 2
    last = {}

    def keep_last(pos, nrm, pixel, depth, it, rho):
        last.update(pos=pos, nrm=nrm, rho=rho.copy())
        return rho

    if mode == "analytic":
        g = _gpu(neb, sc, mode, n_iter)
        o = _oracle(oracle, sc, oracle.OracleScene(sc), mode, n_iter)
    else:
        R = neb.Renderer(sc, flags=neb.FLAG_SINGLE_THREAD_OCTREE)
        R.render(n_iter)
        g = dict(img=R.image_host().astype(np.float64), tech=R.technique_images_host(), stats=R.stats(),
                 octree=R.octree())
        o = oracle.render(sc, n_iter=n_iter, density_hook=keep_last)
        pos = torch.from_numpy(last["pos"].astype(np.float32)).cuda()
        nrm = torch.from_numpy(last["nrm"].astype(np.float32)).cuda()
        rho_g = R.query_density(pos, nrm).cpu().numpy().astype(np.float64)
        R.close()
        ro = last["rho"]
        ratio = np.where(ro > 0, rho_g / np.where(ro > 0, ro, 1.0), np.where(rho_g > 0, np.inf, 1.0))
        off = ~(np.abs(ratio - 1) <= 1e-4)
        print(f"\ndensities at {len(ratio)} NEE vertices: median ratio {np.median(ratio):.7f}, "
              f"{int(off.sum())} beyond 1e-4 (ratios {np.round(ratio[off][:8], 4)})", flush=True)
        assert off.mean() < 1e-3
    terr = technique_errors(g["tech"], o["tech"], n_iter)
    print(f"\nroom 96x96, 2 iterations, {mode}: image {rel_rmse(g['img'], o['mean']):.2e}, techniques {terr}",
          flush=True)
    _counts(g["stats"], o["stats"], lp=False)
    if mode == "octree":
        _octree(g, o)
    for t in ("e", "E"):
        assert terr[t] < TOL, (t, terr[t])


def test_room_96_view_paths(neb, oracle, room96):
    """Every view path of the 96 x 96 room (9216 paths), event by event."""
    g = neb.Renderer(room96, density_mode=neb.DENSITY_ANALYTIC, rho0=ROOM_RHO0, cam_weight=1.0,
                     flags=neb.FLAG_RECORD_PATHS)
    g.render(1)
    rg = g.records()
    g.close()
    ro = oracle.render(room96, n_iter=1, density_mode=oracle.DENSITY_ANALYTIC, rho0=ROOM_RHO0, cam_weight=1.0,
                       record=True, enable_photons=False)["records"]
    frac, same = path_agreement(rg, ro, scene_diag(room96))
    print(f"\nroom 96x96: {frac:.5f} of {len(same)} view paths identical", flush=True)
    assert frac >= 0.999, frac
    # refraction events (type 3) occur: the paths do cross the glass
    assert (rg["type"] == 3).sum() > 100
