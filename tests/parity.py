"""Comparison helpers shared by the GPU parity tests (no test here).

relative RMSE (R22): sqrt(mean over pixels and channels of (I - R)^2) / mean(R).

A technique image is compared element by element with the same measure.
A technique that holds only a sliver of the image (a handful of random
emitter hits, say) is held to the image's tolerance rather than to its own
size: its RMSE is divided by max(mean(R_t), floor * mean(R_total)).
"""
import numpy as np

TECHNIQUES = ("e", "E", "P", "LP")


def rel_rmse(img, ref):
    img = np.asarray(img, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.sqrt(np.mean((img - ref) ** 2)) / np.mean(ref))


def technique_errors(tech_gpu, tech_ref, n_iter, floor=0.01):
    """Element-wise error of every technique image.  tech_gpu: mean images
    (per iteration); tech_ref: the oracle's sums over n_iter iterations.
    Returns {technique: error} (0 where both are zero everywhere, inf where
    only the GPU image is non-zero)."""
    total = sum(np.asarray(tech_ref[t], np.float64) for t in TECHNIQUES if t in tech_ref) / n_iter
    scale_total = floor * float(np.mean(total))
    out = {}
    for t in TECHNIQUES:
        if t not in tech_ref:
            continue
        ref = np.asarray(tech_ref[t], np.float64) / n_iter
        img = np.asarray(tech_gpu[t], np.float64)
        rmse = float(np.sqrt(np.mean((img - ref) ** 2)))
        if not np.any(ref):
            out[t] = 0.0 if not np.any(img) else float("inf")
            continue
        out[t] = rmse / max(float(np.mean(ref)), scale_total)
    return out


def path_agreement(rg, ro, diag, tol=1e-4):
    """Fraction of view paths whose (event type, material) sequences agree
    and whose vertices agree within tol * diag (a primitive swap on a
    shared coplanar edge is allowed), and the per-path mask."""
    same = np.ones(len(rg), bool)
    for k in range(rg.shape[1]):
        a, b = rg[:, k], ro[:, k]
        same &= a["type"] == b["type"]
        live = (a["type"] >= 1) & (a["type"] <= 4)
        same &= ~live | (a["mat"] == b["mat"])
        d = np.linalg.norm(a["pos"].astype(np.float64) - b["pos"], axis=1)
        same &= ~live | (d <= tol * diag)
    return float(same.mean()), same


def scene_diag(sc):
    lo, hi = sc.bbox()
    return float(np.linalg.norm(hi.astype(np.float64) - lo))


def leaf_cells(nodes):
    """Leaf cells of an exported octree node array, keyed by their place in
    the tree (depth, x, y, z at that depth), independent of the order in
    which blocks were allocated: {key: count word}.  A word >= 0 is a leaf
    (count, with a split-failed flag in bit 30), a word < 0 the index of
    the first of eight children (child c = x + 2 y + 4 z)."""
    nodes = np.asarray(nodes)
    out = {}
    stack = [(0, 0, 0, 0, 0)]
    while stack:
        idx, d, x, y, z = stack.pop()
        w = int(nodes[idx])
        if w >= 0:
            out[(d, x, y, z)] = w
            continue
        first = -w
        for c in range(8):
            stack.append((first + c, d + 1, 2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1)))
    return out


def cell_agreement(nodes_a, nodes_b):
    """Fraction of the leaf cells of either tree that the other has with
    the same count."""
    a, b = leaf_cells(nodes_a), leaf_cells(nodes_b)
    keys = set(a) | set(b)
    same = sum(1 for k in keys if a.get(k) == b.get(k))
    return same / max(1, len(keys))
