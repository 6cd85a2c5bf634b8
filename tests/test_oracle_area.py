"""Pins of the oracle's plane-box area (polygon clipping) against facts
that do not depend on it: eq. (area)'s closed special cases (Sec. 5.3),
the volume identity of Appendix A (area = d V / d h, V from the
inclusion-exclusion of simplex volumes, itself checked by Monte Carlo),
additivity over the eight children of a cell, and mirror invariance."""
import numpy as np
import pytest


def _rand_unit(rng):
    n = rng.normal(size=3)
    return n / np.linalg.norm(n)


def test_axis_aligned_normal_gives_face_area(oracle):
    rng = np.random.default_rng(1)
    for _ in range(200):
        lo = rng.uniform(-1, 1, 3)
        hi = lo + rng.uniform(0.01, 2, 3)
        ax = rng.integers(0, 3)
        n = np.zeros(3)
        n[ax] = rng.choice([-1.0, 1.0])
        p = rng.uniform(lo, hi)
        o = [i for i in range(3) if i != ax]
        s = hi - lo
        assert oracle.exact_area(lo, hi, p, n) == pytest.approx(s[o[0]] * s[o[1]], rel=1e-12)


def _chord_2d(lo, hi, p, n):
    """Length of the line {x : n.(x-p)=0} inside the rectangle [lo,hi]
    (Liang-Barsky clipping of the line's parametric form)."""
    d = np.array([-n[1], n[0]])
    d /= np.linalg.norm(d)
    t0, t1 = -np.inf, np.inf
    for i in range(2):
        if abs(d[i]) < 1e-300:
            if p[i] < lo[i] or p[i] > hi[i]:
                return 0.0
            continue
        a, b = (lo[i] - p[i]) / d[i], (hi[i] - p[i]) / d[i]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return max(0.0, t1 - t0)


def test_one_zero_component_reduces_to_chord_times_extent(oracle):
    rng = np.random.default_rng(2)
    for _ in range(300):
        lo = rng.uniform(-1, 1, 3)
        hi = lo + rng.uniform(0.05, 2, 3)
        d = rng.integers(0, 3)
        o = [(d + 1) % 3, (d + 2) % 3]
        n = np.zeros(3)
        ang = rng.uniform(0, 2 * np.pi)
        n[o[0]], n[o[1]] = np.cos(ang), np.sin(ang)
        p = rng.uniform(lo, hi)
        ref = (hi[d] - lo[d]) * _chord_2d(lo[o], hi[o], p[o], n[o])
        assert oracle.exact_area(lo, hi, p, n) == pytest.approx(ref, rel=1e-10, abs=1e-14)


def _volume_below(lo, hi, h, n):
    """Appendix A: volume of {y in box : <n,y> <= h} by inclusion-exclusion
    of simplex volumes, for n with all components > 0."""
    tot = 0.0
    for i in range(8):
        b = np.array([hi[0] if i & 1 else lo[0], hi[1] if i & 2 else lo[1], hi[2] if i & 4 else lo[2]])
        parity = (-1) ** bin(i).count("1")
        tot += parity * max(0.0, h - n @ b) ** 3
    return tot / (6.0 * n[0] * n[1] * n[2])


def test_volume_formula_matches_monte_carlo():
    rng = np.random.default_rng(3)
    for _ in range(5):
        lo = rng.uniform(-1, 0, 3)
        hi = lo + rng.uniform(0.5, 1.5, 3)
        n = np.abs(_rand_unit(rng)) + 0.05
        n /= np.linalg.norm(n)
        p = rng.uniform(lo, hi)
        h = n @ p
        y = rng.uniform(lo, hi, (400000, 3))
        mc = np.prod(hi - lo) * np.mean(y @ n <= h)
        se = np.prod(hi - lo) * 0.5 / np.sqrt(len(y))
        assert abs(_volume_below(lo, hi, h, n) - mc) < 5 * se


def test_area_is_derivative_of_volume(oracle):
    rng = np.random.default_rng(4)
    for _ in range(300):
        lo = rng.uniform(-1, 1, 3)
        hi = lo + rng.uniform(0.1, 2, 3)
        n = _rand_unit(rng)
        if np.min(np.abs(n)) < 0.05:
            continue
        p = rng.uniform(lo, hi)
        # mirror the box so that every normal component is positive
        flo, fhi, fp, fn = lo.copy(), hi.copy(), p.copy(), n.copy()
        for i in range(3):
            if n[i] < 0:
                flo[i], fhi[i], fp[i], fn[i] = -hi[i], -lo[i], -p[i], -n[i]
        h = fn @ fp
        eps = 1e-5 * np.linalg.norm(hi - lo)
        dv = (_volume_below(flo, fhi, h + eps, fn) - _volume_below(flo, fhi, h - eps, fn)) / (2 * eps)
        assert oracle.exact_area(lo, hi, p, n) == pytest.approx(dv, rel=1e-5, abs=1e-9)


def test_additivity_over_children(oracle):
    rng = np.random.default_rng(5)
    for _ in range(200):
        lo = rng.uniform(-1, 1, 3)
        hi = lo + rng.uniform(0.1, 2, 3)
        mid = 0.5 * (lo + hi)
        n = _rand_unit(rng)
        p = rng.uniform(lo, hi)
        parent = oracle.exact_area(lo, hi, p, n)
        kids = 0.0
        for c in range(8):
            clo = np.where([c & 1, c & 2, c & 4], mid, lo)
            chi = np.where([c & 1, c & 2, c & 4], hi, mid)
            kids += oracle.exact_area(clo, chi, p, n)
        assert kids == pytest.approx(parent, rel=1e-9, abs=1e-12)


def test_mirror_invariance_and_bounds(oracle):
    rng = np.random.default_rng(6)
    for _ in range(200):
        lo = rng.uniform(-1, 1, 3)
        hi = lo + rng.uniform(0.1, 2, 3)
        n = _rand_unit(rng)
        p = rng.uniform(lo, hi)
        a = oracle.exact_area(lo, hi, p, n)
        ax = rng.integers(0, 3)
        lo2, hi2, p2, n2 = lo.copy(), hi.copy(), p.copy(), n.copy()
        lo2[ax], hi2[ax], p2[ax], n2[ax] = -hi[ax], -lo[ax], -p[ax], -n[ax]
        assert oracle.exact_area(lo2, hi2, p2, n2) == pytest.approx(a, rel=1e-10)
        assert oracle.exact_area(lo, hi, p, -n) == pytest.approx(a, rel=1e-10)
        s = hi - lo
        # a plane section of a box never exceeds the box's largest diagonal section
        assert a <= np.sqrt((s[0] * s[1]) ** 2 + (s[1] * s[2]) ** 2 + (s[0] * s[2]) ** 2) * (1 + 1e-12)


def test_regular_hexagon_section_of_cube(oracle):
    # the plane through the centre with normal (1,1,1) cuts a regular hexagon of side sqrt(2)/2
    side = np.sqrt(2) / 2
    assert oracle.exact_area([0, 0, 0], [1, 1, 1], [0.5] * 3, [1, 1, 1]) == pytest.approx(
        1.5 * np.sqrt(3) * side ** 2, rel=1e-12)
