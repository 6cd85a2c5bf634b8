"""Pins of the oracle's density octree (Sec. 5 and Appendix B) against the
rules the paper states, worked through by hand on tiny inputs, the
conserved ledger (sum of leaf counts minus 4 x the iteration of every
allocated block equals the number of counted deposits), and the density of
uniformly sampled planes (E[rho] -> points per unit area)."""
import numpy as np
import pytest

from neb_inputs import deposit_stream, plane_deposits

UNIT_LO = np.zeros(3, np.float32)
UNIT_HI = np.ones(3, np.float32)


def test_first_split_follows_the_rules(oracle):
    oc = oracle.Octree(UNIT_LO, UNIT_HI, 64)
    oc.set_iteration(1)                      # threshold 4 * 1, children start at 1
    pts = np.array([[0.2, 0.2, 0.2]] * 4, np.float32)
    oc.increment(pts[:3])
    nodes, info = oc.export()
    assert nodes[0] == 3 and info["allocated"] == 1
    oc.increment(pts[3:])
    nodes, info = oc.export()
    # capacity rounds up to 8n+1; root now points at block 1; 8 children start at 1
    assert info["capacity"] == 65
    assert nodes[0] == -1 and list(nodes[1:9]) == [1] * 8 and info["depth"] == 1
    assert info["ledger"] == 4 == info["deposits"]
    # child index = x_bit + 2*y_bit + 4*z_bit of the first level
    oc.increment(np.array([[0.7, 0.2, 0.9]], np.float32))
    nodes, info = oc.export()
    assert nodes[1 + 5] == 2 and info["ledger"] == 5 == info["deposits"]


def test_threshold_and_child_start_follow_iteration(oracle):
    oc = oracle.Octree(UNIT_LO, UNIT_HI, 64)
    oc.set_iteration(3)                      # threshold 12, children start at 3
    oc.increment(np.array([[0.6, 0.6, 0.6]] * 11, np.float32))
    nodes, _ = oc.export()
    assert nodes[0] == 11
    oc.increment(np.array([[0.6, 0.6, 0.6]], np.float32))
    nodes, info = oc.export()
    assert nodes[0] == -1 and list(nodes[1:9]) == [3] * 8
    assert info["ledger"] == 12 == info["deposits"]
    assert info["block_iter_sum"] == 3


def test_density_of_one_cell(oracle):
    oc = oracle.Octree(UNIT_LO, UNIT_HI, 64)
    oc.set_iteration(1)
    oc.increment(np.array([[0.2, 0.2, 0.2]] * 5, np.float32))   # split at 4, then child 0 -> 2
    size = 1.002
    cell = size / 2
    # horizontal plane through the cell: area = cell^2; rho = count / area (scale 1)
    rho = oc.density_f64([0.2, 0.2, 0.2], [0, 1, 0], robust=False)
    assert rho == pytest.approx(2.0 / cell ** 2, rel=1e-6)
    # two iterations later the same counts are scaled by 1/3
    oc.set_iteration(3)
    assert oc.density_f64([0.2, 0.2, 0.2], [0, 1, 0], robust=False) == pytest.approx(
        2.0 / cell ** 2 / 3, rel=1e-6)


def test_min_area_clamp(oracle):
    oc = oracle.Octree(UNIT_LO, UNIT_HI, 64)
    oc.set_iteration(1)
    oc.increment(np.array([[0.2, 0.2, 0.2]] * 5, np.float32))
    # a plane that only clips a corner of child 0 has a tiny area; the clamp is
    # 1/100 of the squared cell diagonal
    size = 1.002
    diag = np.sqrt(3 * size ** 2) / 2
    lo = -0.001
    corner = np.array([lo, lo, lo]) + 1e-4
    rho = oc.density_f64(corner, np.ones(3) / np.sqrt(3), robust=False)
    assert rho == pytest.approx(2.0 / (0.01 * diag ** 2), rel=1e-5)


@pytest.mark.parametrize("capacity", [1 << 16, 257, 33])
def test_ledger_conservation(oracle, capacity):
    pts = deposit_stream(40000, seed=3)
    oc = oracle.Octree(UNIT_LO, UNIT_HI, capacity)
    total = 0
    for it in range(1, 6):
        oc.set_iteration(it)
        chunk = pts[(it - 1) * 8000: it * 8000]
        oc.increment(chunk)
        total += len(chunk)
        nodes, info = oc.export()
        assert info["ledger"] == info["deposits"] == total
        # structural invariants: pointers land on 8-aligned blocks inside the pool
        ptr = -nodes[nodes < 0]
        assert np.all((ptr - 1) % 8 == 0) and np.all(ptr + 8 <= info["capacity"])
    if capacity < 100:
        assert info["overflow"] > 0


def test_stop_filling_after_1000_iterations(oracle):
    oc = oracle.Octree(UNIT_LO, UNIT_HI, 1024)
    oc.set_iteration(1000)
    oc.increment(deposit_stream(1000, seed=1))
    before, info0 = oc.export()
    oc.set_iteration(1001)
    oc.increment(deposit_stream(1000, seed=2))
    after, info1 = oc.export()
    assert np.array_equal(before, after) and info1["deposits"] == info0["deposits"]


def test_depth_cap(oracle):
    oc = oracle.Octree(UNIT_LO, UNIT_HI, 1 << 12)
    oc.set_iteration(1)
    oc.increment(np.array([[0.3, 0.3, 0.3]] * 2000, np.float32))
    _, info = oc.export()
    assert info["depth"] == 20 and info["ledger"] == info["deposits"] == 2000


def test_out_of_bounds_is_rejected_and_queries_zero(oracle):
    oc = oracle.Octree(UNIT_LO, UNIT_HI, 64)
    oc.set_iteration(1)
    oc.increment(np.array([[1.5, 0.5, 0.5], [-0.2, 0.5, 0.5]], np.float32))
    _, info = oc.export()
    assert info["rejected"] == 2 and info["deposits"] == 0
    assert oc.density_f64([1.5, 0.5, 0.5], [0, 1, 0], robust=False) == 0.0


def _plane_density_error(oracle, normal, offset, n_per_iter, iters, seed):
    oc = oracle.Octree(UNIT_LO, UNIT_HI, 1 << 18)
    nrm = np.asarray(normal, np.float64) / np.linalg.norm(normal)
    for it in range(1, iters + 1):
        oc.set_iteration(it)
        oc.increment(plane_deposits(n_per_iter, seed + it, normal=nrm, offset=offset, lo=0.05, hi=0.95))
    q = plane_deposits(400, seed + 999, normal=nrm, offset=offset, lo=0.15, hi=0.85)
    rho = oc.density(q, np.tile(nrm, (len(q), 1)).astype(np.float32), robust=True)
    # true density: points per unit plane area; the sampled square is 0.9 x 0.9
    # in the two free coordinates, so its plane area is 0.81 / |n_max|
    true = n_per_iter / (0.81 / np.max(np.abs(nrm)))
    return np.median(rho) / true - 1.0, np.mean(np.abs(rho / true - 1.0))


def test_density_of_axis_aligned_plane_converges(oracle):
    err4, _ = _plane_density_error(oracle, (0, 1, 0), 0.437, 20000, 4, seed=10)
    err16, spread16 = _plane_density_error(oracle, (0, 1, 0), 0.437, 20000, 16, seed=10)
    assert abs(err16) < 0.06
    assert abs(err16) <= abs(err4) + 0.02
    assert spread16 < 0.25


def test_density_of_tilted_plane(oracle):
    err, spread = _plane_density_error(oracle, (0.3, 1.0, 0.2), 0.6, 20000, 16, seed=20)
    assert abs(err) < 0.1 and spread < 0.35
