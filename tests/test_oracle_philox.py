"""Pins of the oracle's Philox-4x32-10 against rocRAND's implementation
(compiled on the host from its headers) and a uniformity check of the
24-bit uniforms both sides derive from it."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("philox") / "ref")
    subprocess.run([hipcc, "-O1", "-std=c++17", os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(triples):
        inp = "".join(f"{s} {u} {o}\n" for s, u, o in triples)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()], np.uint64)
    return run


def test_oracle_philox_matches_rocrand(oracle, rocrand_ref):
    rng = np.random.default_rng(0)
    cases = []
    for _ in range(200):
        seed = int(rng.integers(0, 2 ** 63))
        c = [int(x) for x in rng.integers(0, 2 ** 32, 4)]
        sub = c[2] | (c[3] << 32)
        off = 4 * (c[0] | (c[1] << 32) % (2 ** 62))
        c[1] = (off // 4) >> 32
        cases.append((seed, sub, off, c))
    cases.append((0, 0, 0, [0, 0, 0, 0]))
    cases.append((1, 7, 4 * 12345, [12345, 0, 7, 0]))
    ref = rocrand_ref([(s, u, o) for s, u, o, _ in cases])
    for (seed, _, _, c), r in zip(cases, ref):
        mine = oracle.philox(c, [seed & 0xFFFFFFFF, seed >> 32])
        assert list(mine.astype(np.uint64)) == list(r), (seed, c)


def test_uniforms_are_uniform(oracle):
    # chi-square over 64 bins of (x >> 8) * 2^-24 for 40k draws
    vals = []
    for i in range(10000):
        vals.extend(oracle.philox([i, 3, 5, 2], [1, 0]))
    u = (np.asarray(vals, np.uint64) >> 8).astype(np.float64) / 2.0 ** 24
    assert u.min() >= 0.0 and u.max() < 1.0
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    e = len(u) / 64
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 120          # 63 dof, p ~ 1e-5
