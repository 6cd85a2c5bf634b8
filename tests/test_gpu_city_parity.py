"""GPU against the FP64 oracle on the city block's recipe at a small size
(12 x 12 lots, 2036 triangles): glossy GGX boxes (alpha 0.05), a mirror
torus, 64 point lights selected in proportion to their power, path length
10, NEB photons on.

- every view path (48 x 48), event by event;
- 64 iterations, with and without conventional light photons: the image
  and every technique image (E: NEE to point lights, eq. neepdf; P: NEB
  photons, many of them reflected by GGX boxes and the mirror, merged with
  eq. photonpdf; LP: photons from the point lights, eq. stdphotonpdf)
  agree element by element within 1 % relative RMSE (R22), with the
  analytic density and with the single-thread octree; point lights cannot
  be hit, so e is zero on both sides;
- the work counts agree.
"""
import numpy as np
import pytest

from neb_inputs import city_lots
from parity import rel_rmse, technique_errors, path_agreement, scene_diag, cell_agreement

pytestmark = pytest.mark.gpu

RHO0 = 10.0   # NEE vertices per m^2 per iteration, about the octree's level at 48 x 48
TOL = 0.01
N_ITER = 64


@pytest.fixture(scope="module")
def neb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_00573_amd import neb as N
    N.lib()
    return N


@pytest.fixture(scope="module")
def city():
    return city_lots()


def test_city_view_paths(neb, oracle, city):
    g = neb.Renderer(city, density_mode=neb.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0,
                     flags=neb.FLAG_RECORD_PATHS)
    g.render(1)
    rg = g.records()
    g.close()
    ro = oracle.render(city, n_iter=1, density_mode=oracle.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0,
                       record=True, enable_photons=False)["records"]
    frac, same = path_agreement(rg, ro, scene_diag(city))
    print(f"\ncity lots: {frac:.5f} of {len(same)} view paths identical", flush=True)
    assert frac >= 0.999, frac
    # glossy and mirror reflections occur (type 1 scatter at GGX, 2 at the mirror)
    assert (rg["type"] == 2).sum() > 20 and (rg["mat"] == city.materials.shape[0] - 1).sum() > 20


@pytest.mark.parametrize("mode,nlp", [("analytic", 0), ("analytic", 2304), ("octree", 2304)])
def test_city_images_match_oracle(neb, oracle, city, mode, nlp):
    if mode == "analytic":
        g = neb.Renderer(city, density_mode=neb.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0, light_photons=nlp)
        kw = dict(density_mode=oracle.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0)
    else:
        g = neb.Renderer(city, flags=neb.FLAG_SINGLE_THREAD_OCTREE, light_photons=nlp)
        kw = {}
    g.render(N_ITER)
    img = g.image_host().astype(np.float64)
    tech = g.technique_images_host()
    st = g.stats()
    nodes_g = g.octree()[0] if mode == "octree" else None
    g.close()
    o = oracle.render(city, n_iter=N_ITER, light_photons=nlp, **kw)
    err = rel_rmse(img, o["mean"])
    terr = technique_errors(tech, o["tech"], N_ITER)
    so = o["stats"]
    print(f"\ncity lots {mode} n_LP {nlp}: image {err:.2e}, techniques {terr}; photons {st['photons']}/"
          f"{so['photons']:.0f} segments {st['photon_segments']}/{so['photon_segments']:.0f} merges "
          f"{st['merges']}/{so['merges']:.0f} nee_visible {st['nee_visible']}/{so['nee_visible']:.0f}", flush=True)
    if mode == "octree":
        agree = cell_agreement(nodes_g, o["octree"].export()[0])
        print(f"octree leaf cells equal {agree:.5f}", flush=True)
        assert agree > 0.99
    tot = o["sum"].sum()
    assert o["tech"]["e"].sum() == 0 and np.abs(tech["e"]).sum() == 0
    assert o["tech"]["E"].sum() > 0.1 * tot and o["tech"]["P"].sum() > 1e-3 * tot
    if nlp:
        # the point lights hang far above the block: most of their photons
        # leave the scene, and LP carries a small part of the image
        assert o["tech"]["LP"].sum() > 1e-4 * tot
    assert err < TOL, err
    for t, v in terr.items():
        assert v < TOL, (t, v)
    for k in ("vertices", "nee_visible", "photons", "photon_segments"):
        assert st[k] == pytest.approx(so[k], rel=1e-3), k
    assert st["merges"] == pytest.approx(so["merges"], rel=2e-3)
