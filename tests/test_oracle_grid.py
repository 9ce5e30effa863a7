"""Pins of the oracle's grid logic against closed forms, library routines and brute force.

None of these re-types the oracle's own formulas: each check uses an independent
definition (explicit corner enumeration, scipy's morphology, a randomized work-list
closure written with plain loops, dense evaluation, the half-space argument).
"""
import itertools
import random

import numpy as np
import pytest
import scipy.ndimage as ndi

import synth
from oracle import pifu_oracle as O


# ---------------------------------------------------------------- trilinear x2

@pytest.mark.parametrize("coef", [(1, 2, 3, 4), (-3, 5, -7, 2), (0, 0, 1, -1)])
def test_upsample_reproduces_affine_fields_exactly(coef):
    """Trilinear interpolation is exact on affine fields: the interpolated value at
    fine node (i, j, k) equals the field evaluated at coarse coordinate (i/2, j/2, k/2)."""
    a, b, c, d = coef
    n = 6
    I, J, K = np.meshgrid(np.arange(n), np.arange(n + 1), np.arange(n - 2), indexing="ij")
    coarse = a * I + b * J + c * K + d
    fine = O.upsample_x2(coarse)
    fI, fJ, fK = np.meshgrid(np.arange(2 * n - 1), np.arange(2 * n + 1), np.arange(2 * n - 5),
                             indexing="ij")
    expect = a * fI / 2 + b * fJ / 2 + c * fK / 2 + d
    assert fine.shape == expect.shape
    assert np.array_equal(fine, expect)


def test_upsample_binary_gives_dyadic_corner_means():
    """On binary inputs each fine value is the mean over its 1/2/4/8 enclosing coarse
    corners (enumerated explicitly), i.e. an exact multiple of 1/2^m."""
    g = np.random.default_rng(5)
    coarse = (g.random((4, 5, 3)) > 0.5).astype(np.float64)
    fine = O.upsample_x2(coarse)
    for i, j, k in itertools.product(*(range(s) for s in fine.shape)):
        corners = [coarse[a, b, c]
                   for a in sorted({i // 2, (i + 1) // 2})
                   for b in sorted({j // 2, (j + 1) // 2})
                   for c in sorted({k // 2, (k + 1) // 2})]
        assert fine[i, j, k] == sum(corners) / len(corners)


# ---------------------------------------------------------------- dilation

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_neighbourhood26_matches_scipy_binary_dilation(seed):
    g = np.random.default_rng(seed)
    m = g.random((9, 7, 11)) > 0.93
    m[0, 0, 0] = True
    m[-1, -1, -1] = True
    ref = ndi.binary_dilation(m, structure=np.ones((3, 3, 3), bool))
    assert np.array_equal(O.neighbourhood26(m), ref)


# ---------------------------------------------------------------- brute-force localization

def _brute_localize(logit_fn, n0, T, seed):
    """Independent implementation with plain loops and a randomized work list.

    Cube lattices only: level t has n0 * 2^t cells per axis.  Returns per-level
    sets of evaluated (i, j, k) on each level's lattice and the final labels.
    """
    rnd = random.Random(seed)
    cells = n0
    nodes = [(i, j, k) for i in range(cells + 1) for j in range(cells + 1) for k in range(cells + 1)]
    coord = lambda q, c: tuple(-1.0 + 2.0 * x / c for x in q)
    label = {q: int(logit_fn(coord(q, cells)) > 0) for q in nodes}
    done = set(nodes)
    per_level = [set(nodes)]
    for t in range(1, T + 1):
        cells *= 2
        rng_ = range(cells + 1)
        new_label = {}
        interp = {}
        new_done = set()
        for q in itertools.product(rng_, rng_, rng_):
            corners = list(itertools.product(*[sorted({x // 2, (x + 1) // 2}) for x in q]))
            vals = [label[c] for c in corners]
            interp[q] = sum(vals) / len(vals)
            if all(x % 2 == 0 for x in q):
                new_label[q] = label[tuple(x // 2 for x in q)]
                if tuple(x // 2 for x in q) in done:
                    new_done.add(q)
            else:
                new_label[q] = 1 if interp[q] > 0.5 else 0
        nb = lambda q: [(q[0] + a, q[1] + b, q[2] + c) for a in (-1, 0, 1) for b in (-1, 0, 1)
                        for c in (-1, 0, 1)
                        if 0 <= q[0] + a <= cells and 0 <= q[1] + b <= cells and 0 <= q[2] + c <= cells]
        b0 = [q for q in interp if 0 < interp[q] < 1]
        work = sorted({w for q in b0 for w in nb(q) if w not in new_done})
        rnd.shuffle(work)
        queued = set(work)
        evaluated_here = set()
        while work:
            q = work.pop()
            lg = logit_fn(coord(q, cells))
            new_label[q] = int(lg > 0)
            new_done.add(q)
            evaluated_here.add(q)
            if new_label[q] != int(interp[q] > 0.5):
                for w in nb(q):
                    if w not in new_done and w not in queued:
                        queued.add(w)
                        work.insert(rnd.randrange(len(work) + 1), w)
        label = new_label
        done = new_done
        per_level.append(evaluated_here)
    return per_level, label, cells


def _check_against_brute(fld, n0_log2, T, seeds=(0, 1)):
    res = O.occupancy_grid(fld, n0_log2 + T, n0_log2)
    fn = lambda P: float(O.field_logit(fld, np.array([P]))[0])
    for seed in seeds:
        per_level, label, cells = _brute_localize(fn, 1 << n0_log2, T, seed)
        for t, rec in enumerate(res["levels"]):
            n = rec.dims[0]
            got = {(int(x // (n * n)), int((x // n) % n), int(x % n)) for x in rec.evaluated}
            assert got == per_level[t], f"level {t} evaluated sets differ"
        lab = np.zeros((cells + 1,) * 3, np.uint8)
        for q, v in label.items():
            lab[q] = v
        assert np.array_equal(lab, res["labels"])


def test_localization_matches_randomized_worklist_closure_mlp():
    feat = synth.feature_map(16, 16, 8, 2.0, 7)
    mlp = synth.he_mlp(8, 1, [16, 8, 1], [False, False, False], 8)
    _check_against_brute(O.Field("mlp", feat=feat, mlp=mlp), 2, 2)


def test_localization_matches_randomized_worklist_closure_ellipsoids():
    ell = synth.ellipsoids(3, 11, scale=0.6)
    _check_against_brute(O.Field("ellipsoids", ell=ell, sharpness=8.0), 1, 3)


# ---------------------------------------------------------------- invariants

def test_coarsest_equals_final_is_dense():
    feat = synth.tiny_features()
    fld = O.Field("mlp", feat=feat, mlp=synth.tiny_mlp())
    h = O.occupancy_grid(fld, 3, 3)
    d = O.dense_grid(fld, 3)
    assert np.array_equal(h["labels"], d["labels"])
    assert np.array_equal(h["occ"], d["occ"])


@pytest.mark.parametrize("d", [1.0, -1.0])
def test_constant_field_evaluates_only_the_coarse_grid(d):
    fld = O.Field("plane", plane=np.array([0, 0, 0, d]))
    h = O.occupancy_grid(fld, 5, 2)
    assert h["levels"][0].stats["evaluated"] == 5 ** 3
    assert all(r.stats["evaluated"] == 0 for r in h["levels"][1:])
    assert np.all(h["labels"] == (1 if d > 0 else 0))
    assert h["cells"].size == 0


def test_planar_field_equals_dense_everywhere():
    """Inside and outside of a half-space are convex, so a culled node (whose coarse
    corners agree) always has the corners' label: hierarchical == dense at every node."""
    fld = O.Field("plane", plane=synth.PLANE_TINY)
    h = O.occupancy_grid(fld, 5, 2)
    d = O.dense_grid(fld, 5)
    assert np.array_equal(h["labels"], d["labels"])
    assert np.array_equal(h["cells"], d["cells"])
    ev = sum(r.stats["evaluated"] for r in h["levels"])
    assert ev < 33 ** 3 / 2


@pytest.mark.parametrize("seed", [301, 302, 303])
def test_smooth_ellipsoids_surface_cells_match_dense(seed):
    """Ellipsoids resolved at the coarse level: every surface cell of the dense grid is
    found, with identical corner labels (the accuracy claim of Sec. 4.1 / Fig. 3)."""
    fld = O.Field("ellipsoids", ell=synth.ellipsoids(8, seed), sharpness=8.0)
    h = O.occupancy_grid(fld, 6, 3)
    d = O.dense_grid(fld, 6)
    assert np.array_equal(h["cells"], d["cells"])
    n = 64
    ci = d["cells"].astype(np.int64)
    i, j, k = ci // (n * n), (ci // n) % n, ci % n
    for a, b, c in itertools.product((0, 1), repeat=3):
        assert np.array_equal(h["labels"][i + a, j + b, k + c], d["labels"][i + a, j + b, k + c])
    ev = sum(r.stats["evaluated"] for r in h["levels"])
    assert ev < 65 ** 3 / 4


def test_sphere_logit_closed_form():
    """logit = k (1 - |P|^2 / r^2) for a centred sphere (M = I / r, rounded to float32)."""
    r = 0.6
    fld = O.Field("ellipsoids", ell=synth.sphere_as_ellipsoid(r), sharpness=8.0)
    P = np.random.default_rng(0).uniform(-1, 1, (100, 3))
    inv = np.float64(np.float32(1.0 / r))
    assert np.allclose(O.field_logit(fld, P), 8.0 * (1 - np.sum(P * P, axis=1) * inv * inv),
                       rtol=0, atol=1e-12)
    on = np.array([[1, 0, 0], [0, -1, 0], [0, 0, 1.0]]) / inv
    assert np.allclose(O.field_logit(fld, on), 0, atol=1e-12)


def test_surface_cells_bruteforce():
    g = np.random.default_rng(3)
    lab = (g.random((5, 4, 6)) > 0.6).astype(np.uint8)
    cells = []
    for i in range(4):
        for j in range(3):
            for k in range(5):
                v = lab[i:i + 2, j:j + 2, k:k + 2]
                if v.min() != v.max():
                    cells.append((i * 3 + j) * 5 + k)
    assert np.array_equal(O.surface_cells(lab), np.array(cells, np.uint32))
