"""Host checks of the BVH builder (four-wide 128-byte nodes), no device:
every triangle placed once, every stored box holding what lies below it,
closest hits of a nearest-first walk over the tree equal to brute force over
every triangle with the same watertight test, and the walk's deepest stack
within the entries the builder reports (the traversal stack is sized from
that figure)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from neb_inputs import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_00573_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("bvh")
    exe = str(d / "bvh_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "host", "bvh_check.cpp"),
                    os.path.join(CSRC, "neb_bvh.cpp"), "-o", exe], check=True)
    return exe, d


def run(checker, name, vertices, tris, rays):
    exe, d = checker
    path = str(d / (name + ".bin"))
    with open(path, "wb") as f:
        np.array([len(vertices), len(tris)], dtype=np.int32).tofile(f)
        np.ascontiguousarray(vertices, dtype=np.float32).tofile(f)
        np.ascontiguousarray(tris, dtype=np.int32).tofile(f)
    out = subprocess.run([exe, path, str(rays)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (kv.split("=") for kv in out.split())}


def check(r, rays):
    assert r["box_violations"] == 0
    assert r["unseen"] == 0
    assert r["orphans"] == 0
    assert r["rays"] == rays
    assert r["differing"] == 0
    assert r["max_stack"] <= r["stack_need"]


@pytest.mark.parametrize("name", ["tiny_box", "box_room"])
def test_scene_trees(checker, name):
    sc = getattr(scenes, name)()
    r = run(checker, name, sc.vertices, sc.tris, 3000)
    check(r, 3000)
    assert r["hits"] > 2500  # rays start inside closed rooms
    # four-wide: at least a third fewer nodes than the binary tree's n - 1
    assert r["nodes"] < 2 * len(sc.tris) / 3


def test_random_soup(checker):
    v, t = scenes.random_triangle_soup(6000, seed=11)
    r = run(checker, "soup", v, t, 3000)
    check(r, 3000)
    assert r["hits"] > 0


def test_one_triangle_is_a_leaf_root(checker):
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.3]], dtype=np.float32)
    r = run(checker, "one", v, np.array([[0, 1, 2]]), 500)
    check(r, 500)
    assert r["nodes"] == 1 and r["stack_need"] == 0


def test_identical_triangles_split_by_count(checker):
    """Identical centroids cannot be split in space: the builder halves the
    list; the lowest id wins the tie at equal distance."""
    v = np.array([[0, 0, 0], [1, 0, 0.2], [0, 1, 0.5]], dtype=np.float32)
    t = np.tile(np.array([[0, 1, 2]], dtype=np.int32), (40, 1))
    r = run(checker, "same", v, t, 500)
    check(r, 500)
