"""Degenerate and extreme configurations on the GPU against the FP64
oracle (analytic density, so both sides use the same rho):

- path length 1 (only emitters seen directly: no NEE vertex, no photon;
  the camera looks at the ceiling light), 2 (NEE but no NEB merge, which
  needs three segments; light photons still merge at the first vertex)
  and 16 (the largest the library takes);
- a 1 x 1 image and a 7 x 3 image (queues far below one wave, ragged);
- a scene lit only by a point light above an open plane (no emitter can
  be hit, so random hits carry nothing, NEE carries all the light and
  every NEB photon escapes);
- a camera that sees nothing (every path escapes at once);
- an octree whose capacity is the root and one block of children (every
  later split fails, every deposit is still counted: the ledger stays
  exact).
"""
import numpy as np
import pytest

from neb_inputs import tiny_box, point_light_plane
from parity import rel_rmse, technique_errors

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


def _compare(neb, oracle, sc, n_iter=4, tol=0.01, **kw):
    """Image and every technique image compared with the oracle's element
    by element (relative RMSE; a technique holding a sliver of the image
    is held to the image's tolerance, see tests/parity.py)."""
    g = neb.Renderer(sc, density_mode=neb.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0, **kw)
    g.render(n_iter)
    img = g.image_host().astype(np.float64)
    tech = g.technique_images_host()
    st = g.stats()
    g.close()
    o = oracle.render(sc, n_iter=n_iter, density_mode=oracle.DENSITY_ANALYTIC, rho0=RHO0, cam_weight=1.0,
                      **{k: v for k, v in kw.items() if k in ("light_photons",)})
    ref = o["mean"]
    if ref.sum() == 0:
        assert np.abs(img).sum() == 0
    else:
        assert rel_rmse(img, ref) < tol
    for t, v in technique_errors(tech, o["tech"], n_iter).items():
        assert v < tol, (t, v)
    assert st["vertices"] == pytest.approx(o["stats"]["vertices"], rel=2e-3, abs=2)
    return st, o


@pytest.mark.parametrize("L", [1, 2, 16])
def test_path_lengths(neb, oracle, L):
    sc = tiny_box(width=32, height=32, max_path_len=L)
    if L == 1:
        cam = sc.camera.copy()
        cam["eye"], cam["look_at"] = (0.5, 0.3, 0.8), (0.5, 0.999, 0.5)
        sc = sc.with_settings(camera=cam)
    st, o = _compare(neb, oracle, sc, n_iter=4 if L < 16 else 2, light_photons=1024 if L == 2 else 0)
    if L == 1:
        assert st["vertices"] == 0 and st["photons"] == 0 and o["tech"]["e"].sum() > 0
    if L == 2:
        assert o["tech"]["P"].sum() == 0 and o["tech"]["LP"].sum() > 0
    if L == 16:
        assert st["photon_segments"] > 0


@pytest.mark.parametrize("wh", [(1, 1), (7, 3)])
def test_tiny_images(neb, oracle, wh):
    sc = tiny_box().with_settings(width=wh[0], height=wh[1])
    _compare(neb, oracle, sc, n_iter=64)


def test_point_lights_only(neb, oracle):
    sc = point_light_plane(width=16, height_px=16).with_settings(max_path_len=4)
    st, o = _compare(neb, oracle, sc, n_iter=8)
    assert o["tech"]["e"].sum() == 0 and o["tech"]["E"].sum() > 0
    assert st["photons"] > 0 and st["photon_segments"] == 0


def test_camera_sees_nothing(neb, oracle):
    sc = tiny_box(width=16, height=16)
    cam = sc.camera.copy()
    cam["eye"] = (0.5, 0.5, 5.0)        # outside the box, looking away from it
    cam["look_at"] = (0.5, 0.5, 9.0)
    sc = sc.with_settings(camera=cam)
    st, o = _compare(neb, oracle, sc, n_iter=3)
    assert o["sum"].sum() == 0
    assert st["vertices"] == 0 and st["events"] == 0 and st["photons"] == 0
    assert st["paths"] == 3 * 16 * 16


def test_octree_of_one_block(neb):
    sc = tiny_box(width=32, height=32).with_settings(octree_capacity=8)
    g = neb.Renderer(sc)
    g.render(3)
    st = g.stats()
    assert st["oct_capacity"] == 9 and st["oct_allocated"] <= 9
    assert st["oct_overflow"] > 0
    assert st["oct_ledger"] == st["oct_deposits"] == st["vertices"]
    assert np.all(np.isfinite(g.image_host()))
    g.close()
