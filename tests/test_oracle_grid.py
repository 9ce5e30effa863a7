"""Pins of the oracle's grid logic against closed forms, library routines and brute force.

None of these re-types the oracle's own formulas: each check uses an independent
definition (explicit corner enumeration, scipy's morphology, a randomized work-list
closure written with plain loops, dense evaluation, the half-space argument).
"""
import itertools

import numpy as np
import pytest
import scipy.ndimage as ndi

import synth
from oracle import pifu_oracle as O
from brute import brute_localize as _brute_localize


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

def _check_against_brute(fld, n0_log2, T, seeds=(0, 1)):
    res = O.occupancy_grid(fld, n0_log2 + T, n0_log2)
    fn = lambda P: float(O.field_logit(fld, np.array([P]))[0])
    for seed in seeds:
        per_level, label, cells, _, _ = _brute_localize(fn, 1 << n0_log2, T, seed)
        for t, rec in enumerate(res["levels"]):
            n = rec.dims[0]
            got = {(int(x // (n * n)), int((x // n) % n), int(x % n)) for x in rec.evaluated}
            assert got == per_level[t], f"level {t} evaluated sets differ"
        lab = np.zeros(tuple(c + 1 for c in cells), np.uint8)
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


def _check_aniso_against_brute(logit_fn_vec, n0, T, seeds=(0, 1)):
    """O.localize on an anisotropic lattice (the render's: 2^Lw x 2^Lw x 2^Ld cells,
    all axes refined together) against the plain-loop closure."""
    fin = tuple(int(np.log2(c)) + T for c in n0)
    res = O.localize(logit_fn_vec, fin, T)
    fn = lambda P: float(logit_fn_vec(np.array([P]))[0])
    for seed in seeds:
        per_level, label, cells, _, _ = _brute_localize(fn, n0, T, seed)
        for t, rec in enumerate(res.levels):
            nx, ny, nz = rec.dims
            got = {(int(x // (ny * nz)), int((x // nz) % ny), int(x % nz)) for x in rec.evaluated}
            assert got == per_level[t], f"level {t} evaluated sets differ"
        lab = np.zeros(tuple(c + 1 for c in cells), np.uint8)
        for q, v in label.items():
            lab[q] = v
        assert np.array_equal(lab, res.label)
    return res


def test_anisotropic_localization_matches_brute_mlp():
    feat = synth.feature_map(16, 16, 8, 2.0, 7)
    fld = O.Field("mlp", feat=feat, mlp=synth.he_mlp(8, 1, [16, 8, 1], [False] * 3, 8))
    res = _check_aniso_against_brute(lambda P: O.field_logit(fld, P), (4, 4, 2), 2)
    assert res.dims == (17, 17, 9)
    assert sum(r.stats["evaluated"] for r in res.levels[1:]) > 0


@pytest.mark.parametrize("yaw", [0.0, 90.0])
def test_anisotropic_localization_matches_brute_ellipsoids_through_a_view(yaw):
    """The render localizes on its target lattice through the view transform (with the
    clip to the input volume); the closure must be the same on that lattice."""
    # semi-axes scaled 1.5x: some shapes reach past the input volume, so the clip to
    # [-1,1]^3 after the view transform is exercised too
    fld = O.Field("ellipsoids", ell=synth.ellipsoids(4, 12, scale=1.5), sharpness=8.0)
    view = synth.yaw_view(yaw)
    res = _check_aniso_against_brute(lambda P: O.view_logit(fld, view, P), (4, 4, 2), 2,
                                     seeds=(3,))
    assert res.label.any()
    assert all(r.stats["evaluated"] > 0 for r in res.levels)


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


def _ellipsoid_record(c, a, quat_xyzw):
    """A 12-float record (centre, then M = diag(1/a) R^T) built with scipy's rotation
    from a unit quaternion: independent of the input generator's own formula."""
    from scipy.spatial.transform import Rotation
    R = Rotation.from_quat(quat_xyzw).as_matrix()
    M = np.diag(1.0 / np.asarray(a, np.float64)) @ R.T
    return np.concatenate([np.asarray(c, np.float64), M.reshape(-1)]), R


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rotated_offcentre_ellipsoid_closed_form(seed):
    """logit = k (1 - |diag(1/a) R^T (P - c)|^2) for a rotated, off-centre ellipsoid
    (the analytic stand-in): the points c + R diag(a) s u with |u| = 1 give exactly
    k (1 - s^2) -- 0 on the surface, k at the centre.  A transposed M, a sign error in
    the centre or a misplaced semi-axis all move these points off their values."""
    g = np.random.default_rng(seed)
    c = g.uniform(-0.4, 0.4, 3)
    a = np.array([0.2, 0.3, 0.45])[g.permutation(3)]
    q = g.standard_normal(4)
    q /= np.linalg.norm(q)
    rec, R = _ellipsoid_record(c, a, q)
    k = 8.0
    fld = O.Field("ellipsoids", ell=rec[None, :], sharpness=k)
    u = g.standard_normal((200, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    for s in (0.0, 0.5, 1.0, 1.5):
        P = c + (s * u * a) @ R.T
        assert np.allclose(O.field_logit(fld, P), k * (1.0 - s * s), rtol=0, atol=1e-12)
    # the principal axes: c +- a_i R e_i are on the surface, c +- a_i R e_j (j != i,
    # a_j != a_i) are not
    for i in range(3):
        P = c + np.array([a[i] * R[:, i], -a[i] * R[:, i]])
        assert np.allclose(O.field_logit(fld, P), 0.0, atol=1e-12)
        j = (i + 1) % 3
        P = c + a[i] * R[:, j][None, :]
        assert abs(O.field_logit(fld, P)[0]) > 0.1


def test_ellipsoid_union_takes_the_nearest_inside_shape():
    """Union of two disjoint rotated ellipsoids: each one's centre has logit k (the
    minimum of q is 0 there) and a point on either surface, outside the other, has
    logit 0; far points are negative."""
    g = np.random.default_rng(9)
    recs, Rs, cs, As = [], [], [], []
    for c in (np.array([-0.5, 0.1, 0.0]), np.array([0.5, -0.2, 0.1])):
        a = g.uniform(0.1, 0.3, 3)
        q = g.standard_normal(4)
        rec, R = _ellipsoid_record(c, a, q / np.linalg.norm(q))
        recs.append(rec)
        Rs.append(R)
        cs.append(c)
        As.append(a)
    fld = O.Field("ellipsoids", ell=np.stack(recs), sharpness=4.0)
    assert np.allclose(O.field_logit(fld, np.stack(cs)), 4.0, atol=1e-12)
    u = g.standard_normal((50, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    for c, a, R in zip(cs, As, Rs):
        assert np.allclose(O.field_logit(fld, c + (u * a) @ R.T), 0.0, atol=1e-12)
    assert np.all(O.field_logit(fld, np.array([[0.0, 0.9, 0.9], [0.95, 0.95, -0.95]])) < 0)


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
