"""Pins of the oracle's BSDFs, ray casting and explicit MIS densities
against closed forms: Lambert's constant f and cosine pdf, the GGX
normalisation of D cos (Walter et al. 2007), Fresnel at normal incidence
((n-1)/(n+1))^2, Snell's law, the reflection law, an independent
numpy ray-triangle test, cosine-sampling reciprocity (all merge
techniques of an all-Lambertian path have equal density) and the uniform
area density of cosine sampling inside a sphere."""
import numpy as np
import pytest

from neb_inputs import random_triangle_soup, MAT_LAMBERT, MAT_MIRROR, MAT_DIELECTRIC, MAT_GGX


def _unit(rng, n=None):
    v = rng.normal(size=(3,) if n is None else (n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def test_lambert(oracle):
    m = oracle.material(MAT_LAMBERT, (0.2, 0.5, 0.8))
    rng = np.random.default_rng(0)
    for _ in range(200):
        n = _unit(rng)
        wi = _unit(rng)
        ev, d, w, pdf = oracle.bsdf_sample(m, n, wi, rng.uniform(size=3))
        assert ev == 1
        assert np.allclose(w, [0.2, 0.5, 0.8])
        assert np.sign(d @ n) == np.sign(wi @ n)
        f, p = oracle.bsdf_eval(m, n, wi, d)
        assert p == pytest.approx(abs(d @ n) / np.pi, rel=1e-9) == pytest.approx(pdf, rel=1e-9)
        assert np.allclose(f, np.array([0.2, 0.5, 0.8]) / np.pi)
        f2, p2 = oracle.bsdf_eval(m, n, wi, -d)
        assert p2 == 0 and not f2.any()
    # mean cosine of cosine-distributed directions is 2/3
    n = np.array([0, 0, 1.0])
    cs = [oracle.bsdf_sample(m, n, n, rng.uniform(size=3))[1][2] for _ in range(20000)]
    assert np.mean(cs) == pytest.approx(2 / 3, abs=0.01)


@pytest.mark.parametrize("alpha", [0.05, 0.3])
def test_ggx_sampling_consistent_with_eval(oracle, alpha):
    m = oracle.material(MAT_GGX, (1, 1, 1), alpha=alpha)
    rng = np.random.default_rng(1)
    n = np.array([0.0, 1.0, 0.0])
    ok = 0
    ws = []
    for _ in range(500):
        wi = _unit(rng)
        wi[1] = abs(wi[1]) + 0.05
        wi /= np.linalg.norm(wi)
        ev, d, w, pdf = oracle.bsdf_sample(m, n, wi, rng.uniform(size=3))
        if ev == 0:
            continue
        ok += 1
        f, p = oracle.bsdf_eval(m, n, wi, d)
        assert p == pytest.approx(pdf, rel=1e-7)
        assert w[0] == pytest.approx(f[0] * abs(d @ n) / pdf, rel=1e-7)
        assert w[0] > 0
        ws.append(w[0])
        # reciprocity of the pdf's half-vector form
        f_rev, p_rev = oracle.bsdf_eval(m, n, d, wi)
        assert f_rev[0] == pytest.approx(f[0], rel=1e-9)
    assert ok > 350
    # single-scattering microfacet reflection with F = 1 cannot create energy
    assert np.mean(ws) <= 1.0 + 0.02


def test_ggx_distribution_normalised():
    # closed form fact: int D(m) cos(theta_m) d omega_m = 1 (checked by quadrature)
    for alpha in (0.05, 0.3):
        th = np.linspace(0, np.pi / 2, 400001)
        c = np.cos(th)
        a2 = alpha * alpha
        D = a2 / (np.pi * (c * c * (a2 - 1) + 1) ** 2)
        val = np.trapezoid(D * c * np.sin(th), th) * 2 * np.pi
        assert val == pytest.approx(1.0, rel=1e-4)


def test_mirror(oracle):
    m = oracle.material(MAT_MIRROR, (0.9, 0.9, 0.9))
    rng = np.random.default_rng(2)
    for _ in range(100):
        n, wi = _unit(rng), _unit(rng)
        ev, d, w, pdf = oracle.bsdf_sample(m, n, wi, rng.uniform(size=3))
        assert ev == 2 and pdf == 1.0 and np.allclose(w, 0.9)
        assert np.allclose(d, 2 * (wi @ n) * n - wi)


def test_dielectric(oracle):
    m = oracle.material(MAT_DIELECTRIC, (1, 1, 1), ior=1.5)
    n = np.array([0.0, 0.0, 1.0])
    # normal incidence: F = ((1.5 - 1) / (1.5 + 1))^2
    _, p_refl = oracle.bsdf_eval(m, n, n, n)
    assert p_refl == pytest.approx(0.04, rel=1e-12)
    rng = np.random.default_rng(3)
    for _ in range(300):
        wi = _unit(rng)
        ev, d, w, pdf = oracle.bsdf_sample(m, n, wi, rng.uniform(size=3))
        assert np.allclose(w, 1.0)
        entering = wi @ n > 0
        if ev == 2:
            assert np.allclose(d, 2 * (wi @ n) * n - wi)
        else:
            assert ev == 3 and np.sign(d @ n) != np.sign(wi @ n)
            eta = 1 / 1.5 if entering else 1.5
            sin_i = np.linalg.norm(np.cross(wi, n))
            sin_t = np.linalg.norm(np.cross(d, n))
            assert sin_t == pytest.approx(eta * sin_i, rel=1e-9, abs=1e-12)
            # reverse direction has the same lobe probability (Fresnel symmetry)
            _, p_rev = oracle.bsdf_eval(m, n, d, wi)
            assert p_rev == pytest.approx(pdf, rel=1e-9)
    # total internal reflection beyond the critical angle from inside
    th = np.arcsin(1 / 1.5) + 0.05
    wi = np.array([np.sin(th), 0, -np.cos(th)])
    for u0 in (0.0, 0.5, 0.999):
        ev, d, _, pdf = oracle.bsdf_sample(m, n, wi, [u0, 0.3, 0.3])
        assert ev == 2 and pdf == 1.0
    # reflection frequency equals F
    wi = np.array([np.sin(1.0), 0, np.cos(1.0)])
    _, F = oracle.bsdf_eval(m, n, wi, np.array([-wi[0], 0, wi[2]]))
    evs = [oracle.bsdf_sample(m, n, wi, [u, 0.5, 0.5])[0] for u in np.linspace(0, 1, 2001)[:-1]]
    assert np.mean(np.array(evs) == 2) == pytest.approx(F, abs=1e-3)


def _np_closest(v, t, o, d):
    best, prim = np.inf, -1
    for i, (a, b, c) in enumerate(t):
        p0, p1, p2 = v[a].astype(np.float64), v[b].astype(np.float64), v[c].astype(np.float64)
        nn = np.cross(p1 - p0, p2 - p0)
        den = nn @ d
        if den == 0:
            continue
        tt = nn @ (p0 - o) / den
        if tt <= 0:
            continue
        x = o + tt * d
        # inside test with signed areas
        s0 = np.cross(p1 - p0, x - p0) @ nn
        s1 = np.cross(p2 - p1, x - p1) @ nn
        s2 = np.cross(p0 - p2, x - p2) @ nn
        if (s0 >= 0 and s1 >= 0 and s2 >= 0) and tt < best:
            best, prim = tt, i
    return prim, best


def test_closest_hit_matches_independent_test(oracle):
    from neb_inputs.scenes import Scene, _materials, _camera, _no_lights
    v, t = random_triangle_soup(60, seed=4)
    sc = Scene("soup", v, t, np.zeros(len(t), np.int32), _materials([{"albedo": (0.5,) * 3}]),
               _no_lights(), _camera([0, 0, 0], [0, 0, -1]))
    osc = oracle.OracleScene(sc)
    rng = np.random.default_rng(5)
    hits = 0
    for _ in range(400):
        o = rng.uniform(-0.5, 1.5, 3)
        if rng.uniform() < 0.7:      # aim at a jittered triangle centroid
            tgt = v[t[rng.integers(0, len(t))]].mean(axis=0) + rng.normal(0, 0.05, 3)
            d = (tgt - o) / np.linalg.norm(tgt - o)
        else:
            d = _unit(rng)
        prim, tt = osc.closest_hit(o, d)
        rp, rt = _np_closest(v, t, o, d)
        assert prim == rp
        if prim >= 0:
            hits += 1
            assert tt == pytest.approx(rt, rel=1e-9)
    assert hits > 150


def test_closest_hit_inside_box(oracle):
    from neb_inputs import tiny_box
    osc = oracle.OracleScene(tiny_box())
    prim, t = osc.closest_hit([0.2, 0.3, 0.4], [0.0, -1.0, 0.0])
    assert t == pytest.approx(0.3, rel=1e-12) and prim in (0, 1)
    prim, t = osc.closest_hit([0.2, 0.3, 0.4], [1.0, 0.0, 0.0])
    assert t == pytest.approx(0.8, rel=1e-12) and prim in (6, 7)


def test_mis_technique_count_and_reciprocity(oracle):
    """A path of length l has one random hit, one NEE (l >= 2) and l-2
    merge techniques (Sec. 4).  For Lambertian vertices the forward and
    reverse area densities of every segment agree (cos cos / (pi d^2)),
    so all merge techniques have the same density."""
    lam = oracle.material(MAT_LAMBERT, (0.5, 0.5, 0.5))
    rng = np.random.default_rng(6)
    for L in range(1, 8):
        # a zig-zag path between two parallel planes, camera above
        pos = [np.array([0.0, 1.5, 0.0])]
        nrm = [np.array([0.0, -1.0, 0.0])]
        for i in range(1, L + 1):
            y = 0.0 if i % 2 else 1.0
            pos.append(np.array([rng.uniform(-1, 1), y, rng.uniform(-1, 1)]))
            nrm.append(np.array([0.0, 1.0 if y == 0.0 else -1.0, 0.0]))
        pd = oracle.technique_densities(np.array(pos), np.array(nrm), [lam] * max(0, L - 1),
                                        p_light=0.3, hittable=True, rho=50.0, radius=0.01)
        assert len(pd) == 2 + max(0, L - 2)
        assert pd[0] > 0 and (pd[1] > 0) == (L >= 2)
        if L >= 4:
            assert np.allclose(pd[2:], pd[2], rtol=1e-9)


def test_mis_densities_inside_a_sphere(oracle):
    """Cosine sampling between points of a sphere of radius R has area
    density 1/(4 pi R^2); with a uniform area light on the sphere all
    of e, E coincide and every merge technique equals p_l rho pi r^2
    times the same power."""
    lam = oracle.material(MAT_LAMBERT, (0.5, 0.5, 0.5))
    rng = np.random.default_rng(7)
    R = 1.7
    for L in range(2, 7):
        pts = _unit(rng, L) * R
        pos = np.vstack([[0.0, 0.0, 0.0], pts])
        nrm = -pos / R
        nrm[0] = [0, 0, 1]
        pl = 1.0 / (4 * np.pi * R * R)
        rho, r = 30.0, 0.02
        pd = oracle.technique_densities(pos, nrm, [lam] * (L - 1), p_light=pl, hittable=True,
                                        rho=rho, radius=r)
        # p_{0->1} is dropped: e has L-1 segment densities, E has L-2
        a = 1.0 / (4 * np.pi * R * R)
        assert pd[0] == pytest.approx(a ** (L - 1), rel=1e-9)
        assert pd[1] == pytest.approx(pl * a ** (L - 2), rel=1e-9)
        for k in range(1, L - 1):
            assert pd[1 + k] == pytest.approx(pl * rho * np.pi * r * r * a ** (L - 2), rel=1e-9)


def test_mis_caustic_path_has_only_random_hit_and_first_merge(oracle):
    """camera -> diffuse floor -> glass -> glass -> light: NEE at a delta
    vertex and merges at delta vertices are impossible."""
    lam = oracle.material(MAT_LAMBERT, (0.5, 0.5, 0.5))
    glass = oracle.material(MAT_DIELECTRIC, (1, 1, 1), ior=1.5)
    # build a physically consistent refraction chain through a slab y in [0.4, 0.5]
    n_up = np.array([0.0, 1.0, 0.0])
    x1 = np.array([0.0, 0.0, 0.0])
    d1 = np.array([0.3, 1.0, 0.1]); d1 /= np.linalg.norm(d1)
    x2 = x1 + d1 * (0.4 / d1[1])
    eta = 1 / 1.5
    c = -(-d1) @ (-n_up)
    # refraction of the incoming ray (travelling d1) entering through the bottom face (normal -y)
    wi = -d1
    ns = -n_up
    ci = wi @ ns
    ct = np.sqrt(1 - eta * eta * (1 - ci * ci))
    d2 = -eta * wi + (eta * ci - ct) * ns
    x3 = x2 + d2 * (0.1 / d2[1])
    wi = -d2
    ns = n_up * -1 if wi @ n_up < 0 else n_up
    ci = abs(wi @ n_up)
    eta = 1.5
    ct = np.sqrt(1 - eta * eta * (1 - ci * ci))
    d3 = -eta * wi + (eta * ci - ct) * (-n_up)
    x4 = x3 + d3 * (0.5 / d3[1])
    pos = np.array([[0, 2.0, -1.0], x1, x2, x3, x4])
    nrm = np.array([[0, 0, 1.0], n_up, -n_up, n_up, -n_up])
    del c
    pd = oracle.technique_densities(pos, nrm, [lam, glass, glass], p_light=0.5, hittable=True,
                                    rho=10.0, radius=0.01)
    assert pd[0] > 0 and pd[2] > 0          # e and P_1
    assert pd[1] == 0 and pd[3] == 0        # E and P_2
