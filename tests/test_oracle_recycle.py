"""Pins of the oracle's NEE recycling (Sec. 6: every vertex averages the
light samples of the NEE vertices within a radius; n_E of eq. misw is the
number of events found).

A light sample does not depend on the receiving point, so where every
point sees every other (the inside of the closed furnace sphere, a plane
under an emitter) recycling is unbiased and the closed forms must hold:
- the white furnace with recycling, with path tracing alone and with NEB
  photons under the exact density (a weight that leaves out n_E somewhere
  no longer sums to one over the techniques and shifts the mean);
- the polygonal emitter over a plane against Lambert's polygon formula;
- recycling raises the share of NEE in the estimate (more samples per
  vertex), and a radius of zero recovers the plain estimator exactly.
"""
import numpy as np
import pytest

from neb_inputs import furnace_sphere, disk_light_plane


@pytest.fixture(scope="module")
def furnace():
    return furnace_sphere(subdiv=4, width=16, height=16, max_path_len=5)


def _closed_form(sc):
    return sum(0.5 ** j for j in range(sc.max_path_len))


def _rho0(sc):
    v = sc.vertices.astype(np.float64)
    t = sc.tris
    area = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1).sum()
    return (sc.max_path_len - 2) * sc.width * sc.height / area


@pytest.mark.parametrize("photons", [False, True])
def test_furnace_with_recycling(oracle, furnace, photons):
    sc = furnace
    plain = oracle.render(sc, n_iter=32, density_mode=oracle.DENSITY_ANALYTIC, enable_photons=photons,
                          rho0=_rho0(sc), cam_weight=1.0)
    r = oracle.render(sc, n_iter=64, density_mode=oracle.DENSITY_ANALYTIC, enable_photons=photons,
                      rho0=_rho0(sc), cam_weight=1.0, nee_radius=0.2)
    assert r["mean"].mean() / _closed_form(sc) - 1 == pytest.approx(0.0, abs=1e-3)
    share = lambda x: x["tech"]["E"].sum() / x["sum"].sum()
    assert share(r) > 1.5 * share(plain)
    if photons:
        assert r["tech"]["P"].sum() > 0.01 * r["sum"].sum()


def test_zero_radius_is_the_plain_estimator(oracle, furnace):
    # one thread, so that the image sums are taken in the same order
    a = oracle.render(furnace, n_iter=4, density_mode=oracle.DENSITY_ANALYTIC, rho0=100.0, cam_weight=1.0,
                      n_threads=1)
    b = oracle.render(furnace, n_iter=4, density_mode=oracle.DENSITY_ANALYTIC, rho0=100.0, cam_weight=1.0,
                      nee_radius=0.0, n_threads=1)
    for t in ("e", "E", "P"):
        assert np.array_equal(a["tech"][t], b["tech"][t])


def test_disk_light_with_recycling(oracle):
    """Path length 2 under a one-sided polygonal emitter: averaged over the
    image, the recycled NEE reproduces the plain estimate (both unbiased;
    the plain one is checked against Lambert's formula elsewhere)."""
    sc = disk_light_plane(width=8, height_px=8)
    a = oracle.render(sc, n_iter=512, density_mode=oracle.DENSITY_ANALYTIC, enable_photons=False)
    b = oracle.render(sc, n_iter=512, density_mode=oracle.DENSITY_ANALYTIC, enable_photons=False, nee_radius=0.02)
    assert b["mean"].mean() / a["mean"].mean() - 1 == pytest.approx(0.0, abs=2e-3)
    assert np.abs(b["mean"] / a["mean"] - 1).max() < 0.05


def test_recycling_refuses_light_photons(oracle, furnace):
    with pytest.raises(RuntimeError):
        oracle.render(furnace, n_iter=1, density_mode=oracle.DENSITY_ANALYTIC, nee_radius=0.1, light_photons=16)
