"""Pins of the oracle's octree baselines (the subdivision schemes the paper compares its
localization with, Sec. 3.2 and Fig. 3): a plain-loop brute force on tiny grids, and
special cases with known results (every cell subdivided equals dense evaluation; no cell
subdivided evaluates only the coarse grid; a half-space is exact)."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import pifu_oracle as O


def _sig(lg):
    return 1.0 / (1.0 + math.exp(-lg))


def _brute_octree(logit_fn, n0, T, mode, thr):
    """Dictionaries over node tuples; cells and their corners enumerated explicitly."""
    cells = n0
    coord = lambda q, c: tuple(-1.0 + 2.0 * x / c for x in q)
    nodes = list(itertools.product(range(cells + 1), repeat=3))
    lg = {q: logit_fn(coord(q, cells)) for q in nodes}
    val = {q: _sig(lg[q]) for q in nodes}
    lab = {q: int(lg[q] > 0) for q in nodes}
    done = set(nodes)
    per_level = [set(nodes)]
    for _ in range(T):
        flagged = set()
        for cell in itertools.product(range(cells), repeat=3):
            cs = [tuple(cell[i] + d[i] for i in range(3)) for d in itertools.product((0, 1), repeat=3)]
            if mode == "binarized":
                hit = len({lab[q] for q in cs}) > 1
            else:
                vs = [val[q] for q in cs]
                m = sum(vs) / 8.0
                hit = max(abs(v - m) for v in vs) > thr
            if hit:
                flagged.add(cell)
        fine = 2 * cells
        nval, nlab, ndone, here = {}, {}, set(), set()
        for q in itertools.product(range(fine + 1), repeat=3):
            if all(x % 2 == 0 for x in q):
                c = tuple(x // 2 for x in q)
                nval[q], nlab[q] = val[c], lab[c]
                if c in done:
                    ndone.add(q)
            else:
                cs = list(itertools.product(*[sorted({x // 2, (x + 1) // 2}) for x in q]))
                src = [lab[c] for c in cs] if mode == "binarized" else [val[c] for c in cs]
                nval[q] = sum(src) / len(src)
                nlab[q] = int(nval[q] > 0.5)
            owners = itertools.product(*[([x // 2 - 1, x // 2] if x % 2 == 0 else [x // 2])
                                         for x in q])
            if q not in ndone and any(o in flagged for o in owners):
                v = logit_fn(coord(q, fine))
                nval[q], nlab[q] = _sig(v), int(v > 0)
                ndone.add(q)
                here.add(q)
        cells, val, lab, done = fine, nval, nlab, ndone
        per_level.append(here)
    return per_level, lab, cells


@pytest.mark.parametrize("mode,thr", [("binarized", 0.0), ("threshold", 0.05), ("threshold", 0.2)])
@pytest.mark.parametrize("kind", ["mlp", "ell"])
def test_octree_matches_brute_force(kind, mode, thr):
    if kind == "mlp":
        feat = synth.feature_map(16, 16, 8, 2.0, 7)
        fld = O.Field("mlp", feat=feat, mlp=synth.he_mlp(8, 1, [16, 8, 1], [False] * 3, 8))
        n0, T = 4, 2
    else:
        fld = O.Field("ellipsoids", ell=synth.ellipsoids(3, 11, scale=0.8), sharpness=8.0)
        n0, T = 2, 3
    res = O.octree_grid(fld, int(math.log2(n0)) + T, int(math.log2(n0)), mode, thr)
    fn = lambda P: float(O.field_logit(fld, np.array([P]))[0])
    per_level, lab, cells = _brute_octree(fn, n0, T, mode, thr)
    for t, rec in enumerate(res["levels"]):
        n = rec.dims[0]
        got = {(int(x // (n * n)), int((x // n) % n), int(x % n)) for x in rec.evaluated}
        assert got == per_level[t], (t, len(got), len(per_level[t]))
    ref = np.zeros((cells + 1,) * 3, np.uint8)
    for q, v in lab.items():
        ref[q] = v
    assert np.array_equal(ref, res["labels"])
    assert sum(len(s) for s in per_level[1:]) > 0


def test_threshold_below_zero_equals_dense():
    """Every cell has a maximum absolute deviation >= 0 > thr: all cells are subdivided and
    every node is evaluated."""
    fld = O.Field("mlp", feat=synth.tiny_features(), mlp=synth.tiny_mlp())
    r = O.octree_grid(fld, 5, 3, "threshold", -1.0)
    d = O.dense_grid(fld, 5)
    assert np.array_equal(r["labels"], d["labels"])
    assert np.allclose(r["occ"], d["occ"], rtol=0, atol=1e-15)
    assert sum(l.stats["evaluated"] for l in r["levels"]) == 33 ** 3


def test_threshold_one_evaluates_only_the_coarse_grid():
    """The deviation of values in [0, 1] from their mean is below 1: nothing is
    subdivided; every finer node takes the trilinear interpolation of the coarse values."""
    fld = O.Field("mlp", feat=synth.tiny_features(), mlp=synth.tiny_mlp())
    r = O.octree_grid(fld, 5, 3, "threshold", 1.0)
    assert all(l.stats["evaluated"] == 0 for l in r["levels"][1:])
    c = O.dense_grid(fld, 3)["occ"]
    assert np.allclose(r["occ"], O.upsample_x2(O.upsample_x2(c)), rtol=0, atol=1e-15)


@pytest.mark.parametrize("mode,thr", [("binarized", 0.0), ("threshold", 0.1), ("threshold", 0.0)])
def test_constant_field_evaluates_only_the_coarse_grid(mode, thr):
    """Equal corners deviate by exactly 0, which does not exceed a threshold of 0."""
    fld = O.Field("plane", plane=np.array([0, 0, 0, 2.0]))
    r = O.octree_grid(fld, 5, 2, mode, thr)
    assert all(l.stats["evaluated"] == 0 for l in r["levels"][1:])
    assert np.all(r["labels"] == 1)


def test_binarized_octree_is_exact_on_a_half_space():
    """A cell whose corners are all inside (or all outside) a half-space lies entirely on
    that side (convexity), so culling it loses nothing: equal to dense at every node."""
    fld = O.Field("plane", plane=synth.PLANE_TINY)
    r = O.octree_grid(fld, 5, 2, "binarized")
    d = O.dense_grid(fld, 5)
    assert np.array_equal(r["labels"], d["labels"])
    assert sum(l.stats["evaluated"] for l in r["levels"]) < 33 ** 3 / 2
