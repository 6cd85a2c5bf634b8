"""Pins of the oracle's conventional light photons (the optional technique
of Sec. 4, eq. stdphotonpdf, weighted by eq. misw).

- technique densities inside a sphere, where cosine sampling and an area
  light on the sphere (or a point light at its centre) give the closed
  form a = 1 / (4 pi R^2) per segment, so LP_k = n_LP p_l pi r^2 a^(L-1)
  for every k;
- technique densities of an open path with a GGX vertex, assembled by hand
  from the BSDF pdfs and the geometry (pins which pdfs enter LP_k, the
  emission density of an area and of a point light, and that LP_{L-1}
  takes the forward pdfs only);
- the white furnace: light photons alone with random hits and NEE, and
  together with NEB photons under the exact density, reproduce the
  closed-form radiance (a wrong flux, emission distribution or weight
  that does not sum to one across techniques shifts the mean);
- a plane under a point light, where light photons carry almost all of the
  weight, against the analytic irradiance (the only bias left is the
  blur of the merge disc, about -0.2 % here).
"""
import numpy as np
import pytest

from neb_inputs import furnace_sphere, point_light_plane

MAT_LAMBERT, MAT_GGX = 0, 3


def _unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("hittable", [True, False])
def test_lp_densities_inside_a_sphere(oracle, hittable):
    lam = oracle.material(MAT_LAMBERT, (0.5, 0.5, 0.5))
    rng = np.random.default_rng(17)
    R, rho, r, n_lp, pl = 1.3, 25.0, 0.03, 1000.0, 0.7
    a = 1.0 / (4 * np.pi * R * R)
    for L in range(2, 7):
        if hittable:
            pts = _unit(rng, L) * R
            pos = np.vstack([[0.0, 0.0, 0.0], pts])
            nrm = -pos / R
        else:
            # the last vertex is a point light at the centre
            pts = _unit(rng, L - 1) * R
            pos = np.vstack([[0.0, 0.0, 0.0], pts, [[0.0, 0.0, 0.0]]])
            nrm = np.vstack([-pos[:-1] / R, [[1.0, 0.0, 0.0]]])
        nrm[0] = [0, 0, 1]
        pd = oracle.technique_densities(pos, nrm, [lam] * (L - 1), p_light=pl, hittable=hittable,
                                        rho=rho, radius=r, n_lp=n_lp)
        assert len(pd) == 2 + (L - 2) + (L - 1)
        lp = pd[2 + (L - 2):]
        assert np.allclose(lp, n_lp * pl * np.pi * r * r * a ** (L - 1), rtol=1e-9, atol=0)
        # without light photons the LP entries are zero and the rest is unchanged
        pd0 = oracle.technique_densities(pos, nrm, [lam] * (L - 1), p_light=pl, hittable=hittable,
                                         rho=rho, radius=r, n_lp=0.0)
        assert np.all(pd0[2 + (L - 2):] == 0) and np.allclose(pd0[:2 + (L - 2)], pd[:2 + (L - 2)], rtol=0)


def _toward(a, b):
    d = b - a
    d2 = d @ d
    return d / np.sqrt(d2), d2


@pytest.mark.parametrize("hittable", [True, False])
def test_lp_densities_open_path_by_hand(oracle, hittable):
    """camera x0 -> GGX floor x1 -> Lambert wall x2 -> light x3."""
    ggx = oracle.material(MAT_GGX, (0.8, 0.8, 0.8), alpha=0.3)
    lam = oracle.material(MAT_LAMBERT, (0.5, 0.5, 0.5))
    x = np.array([[0.0, 1.5, 0.0], [0.1, 0.0, 0.05], [1.0, 0.7, 0.3], [0.4, 1.2, -0.2]])
    n = np.array([[0, 0, 1.0], [0, 1.0, 0], [-1.0, 0, 0], [0, -1.0, 0]])
    pl, rho, r, n_lp = 2.0, 40.0, 0.02, 5000.0
    pd = oracle.technique_densities(x, n, [ggx, lam], p_light=pl, hittable=hittable, rho=rho,
                                    radius=r, n_lp=n_lp)
    assert len(pd) == 2 + 1 + 2
    w01, _ = _toward(x[1], x[0])
    w12, d12 = _toward(x[1], x[2])
    w23, d23 = _toward(x[2], x[3])
    # forward (camera-side) densities p_{i -> i+1}, area measure at x_{i+1}
    _, pdf1 = oracle.bsdf_eval(ggx, n[1], w01, w12)
    f1 = pdf1 * abs(n[2] @ w12) / d12
    _, pdf2 = oracle.bsdf_eval(lam, n[2], -w12, w23)
    f2 = pdf2 * abs(n[3] @ w23) / d23
    # reverse density p_{2 -> 1}: sampling at x2 from the light side toward x1
    _, pdf2r = oracle.bsdf_eval(lam, n[2], w23, -w12)
    r1 = pdf2r * abs(n[1] @ w12) / d12
    # emission density p_{3 -> 2}
    emit = max(0.0, -(n[3] @ w23)) / np.pi if hittable else 1.0 / (4 * np.pi)
    rl = emit * abs(n[2] @ w23) / d23
    disc = np.pi * r * r
    assert pd[0] == pytest.approx(f1 * f2 if hittable else 0.0, rel=1e-12, abs=0)
    assert pd[1] == pytest.approx(pl * f1, rel=1e-12)
    assert pd[2] == pytest.approx(pl * rho * disc * r1, rel=1e-12)
    assert pd[3] == pytest.approx(n_lp * pl * disc * rl * r1, rel=1e-12)
    assert pd[4] == pytest.approx(n_lp * pl * disc * rl * f1, rel=1e-12)
    # the GGX lobe makes the two merge positions differ
    assert abs(pd[3] / pd[4] - 1) > 0.1


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


def test_furnace_light_photons_without_neb_photons(oracle, furnace):
    sc = furnace
    r = oracle.render(sc, n_iter=64, density_mode=oracle.DENSITY_ANALYTIC, enable_photons=False,
                      light_photons=256)
    assert r["tech"]["P"].sum() == 0
    assert r["tech"]["LP"].sum() > 0.03 * r["sum"].sum()
    assert r["stats"]["light_photons"] == 64 * 256
    assert r["mean"].mean() / _closed_form(sc) - 1 == pytest.approx(0.0, abs=1e-3)


def test_furnace_neb_and_light_photons_with_exact_density(oracle, furnace):
    sc = furnace
    r = oracle.render(sc, n_iter=64, density_mode=oracle.DENSITY_ANALYTIC, enable_photons=True,
                      rho0=_rho0(sc), cam_weight=1.0, light_photons=256)
    tot = r["sum"].sum()
    assert r["tech"]["P"].sum() > 0.03 * tot and r["tech"]["LP"].sum() > 0.03 * tot
    assert r["mean"].mean() / _closed_form(sc) - 1 == pytest.approx(0.0, abs=1e-3)


def test_point_light_plane_light_photons(oracle):
    sc = point_light_plane()
    r = oracle.render(sc, n_iter=256, density_mode=oracle.DENSITY_ANALYTIC, enable_photons=False,
                      light_photons=262144)
    assert r["tech"]["e"].sum() == 0
    assert r["tech"]["LP"].sum() > 0.95 * r["sum"].sum()
    img = r["mean"][..., 0]
    cam = sc.camera
    th = np.tan(np.radians(float(cam["vfov_deg"])) / 2)
    h = float(sc.point_lights["pos"][0, 1])
    inten = float(sc.point_lights["power"][0, 0]) / (4 * np.pi)
    alb = float(sc.materials["albedo"][0, 0])
    W, H, sub = sc.width, sc.height, 8
    ref = np.zeros((H, W))
    s = (np.arange(sub) + 0.5) / sub
    for py in range(H):
        for px in range(W):
            u = (px + s[None, :]) / W
            v = (py + s[:, None]) / H
            X = (2 * u - 1) * th * (h / 2)       # the camera is h/2 above the plane
            Z = (1 - 2 * v) * th * (h / 2)
            d2 = X * X + Z * Z + h * h
            ref[py, px] = np.mean(alb / np.pi * inten * h / d2 ** 1.5)
    assert img.mean() / ref.mean() - 1 == pytest.approx(-0.002, abs=3e-3)
    assert np.abs(img / ref - 1).max() < 0.03
