"""Pins of the oracle's mesh hand-off (Marching Cubes over the surface cells, the PIFu
baseline's extraction; Sec. 1, Sec. 3.2): the derived table uses exactly the crossing
edges of each case; the mesh is closed and consistently oriented on random labellings
(so ambiguous faces are cut alike by neighbouring cells); a sphere gives Euler
characteristic 2 and its volume; an affine occupancy gives vertices on its plane and the
plane section's area; front-facing vertices of a sphere are the visible ones."""
import math
from collections import Counter

import numpy as np
import pytest

import synth
from oracle import pifu_oracle as O


def test_each_case_uses_exactly_its_crossing_edges():
    for case in range(256):
        tris = O.mc_case_triangles(case)
        used = {e for t in tris for e in t}
        cross = set()
        for e in range(12):
            a, b = O._mc_edge_corners(e)
            if ((case >> a) & 1) != ((case >> b) & 1):
                cross.add(e)
        assert used == cross, case
        assert all(len(set(t)) == 3 for t in tris)
    assert O.mc_case_triangles(0) == [] and O.mc_case_triangles(255) == []


def _edges(tris):
    return Counter((int(t[a]), int(t[(a + 1) % 3])) for t in tris for a in range(3))


def _on_grid_boundary(g1, g2, n):
    """Both vertices' edges lie on one outer face of the node grid."""
    def face_coords(g):
        axis, node = g % 3, g // 3
        q = [node // (n * n), (node // n) % n, node % n]
        out = set()
        for ax in range(3):
            if ax == axis:
                continue
            if q[ax] == 0:
                out.add((ax, 0))
            if q[ax] == n - 1:
                out.add((ax, 1))
        return out
    return bool(face_coords(g1) & face_coords(g2))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_labellings_give_a_closed_oriented_mesh(seed):
    rng = np.random.default_rng(seed)
    n = 7
    lab = (rng.random((n, n, n)) < 0.45).astype(np.uint8)
    occ = np.where(lab == 1, rng.uniform(0.5001, 1.0, lab.shape), rng.uniform(0.0, 0.5, lab.shape))
    m = O.mesh_from_grid(occ, lab)
    cnt = _edges(m["tris"])
    ids = m["edge_ids"]
    for (a, b), c in cnt.items():
        assert c == 1, (a, b, c)           # no edge traversed twice the same way
        if (b, a) not in cnt:
            assert _on_grid_boundary(int(ids[a]), int(ids[b]), n), (a, b)
    # every vertex is used
    assert set(np.unique(m["tris"])) == set(range(ids.size))


def test_sphere_is_closed_genus_zero_with_its_volume():
    r = 0.6
    ell = np.array([[0.0, 0.0, 0.0, 1 / r, 0, 0, 0, 1 / r, 0, 0, 0, 1 / r]], np.float32)
    g = O.dense_grid(O.Field("ellipsoids", ell=ell, sharpness=8.0), 5)
    m = O.mesh_from_grid(g["occ"], g["labels"])
    V, F = m["verts"].shape[0], m["tris"].shape[0]
    E = len({tuple(sorted(e)) for e in _edges(m["tris"])})
    assert V - E + F == 2
    v = m["verts"][m["tris"]]
    vol = float(np.sum(np.einsum("ij,ij->i", v[:, 0], np.cross(v[:, 1], v[:, 2])))) / 6.0
    assert vol > 0
    assert vol == pytest.approx(4.0 / 3.0 * math.pi * r ** 3, rel=0.03)


def test_affine_occupancy_gives_the_plane_section():
    n = 17
    x = np.linspace(-1, 1, n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    nrm = np.array([0.2, -0.3, 1.0])
    d = 0.1
    s = nrm[0] * X + nrm[1] * Y + nrm[2] * Z - d
    occ = 0.5 + 0.2 * s           # stays inside (0, 1) on the grid
    lab = (occ > 0.5).astype(np.uint8)
    m = O.mesh_from_grid(occ, lab)
    P = m["verts"]
    assert np.max(np.abs(P @ nrm - d)) < 1e-12
    v = P[m["tris"]]
    area = 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1).sum()
    # the plane meets every vertical line of [-1, 1]^2 inside the cube
    assert area == pytest.approx(4.0 * np.linalg.norm(nrm) / abs(nrm[2]), rel=1e-12)
    normals = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    # occupancy grows along nrm: outward (towards label 0) is -nrm (triangles of zero
    # area, where a vertex falls on a node, have no direction)
    big = np.linalg.norm(normals, axis=1) > 1e-12
    assert np.all(normals[big] @ nrm < 0) and np.all(normals @ nrm <= 1e-15)


def test_front_vertices_of_a_sphere_are_visible():
    r = 0.6
    ell = np.array([[0.1, -0.1, 0.0, 1 / r, 0, 0, 0, 1 / r, 0, 0, 0, 1 / r]], np.float32)
    g = O.dense_grid(O.Field("ellipsoids", ell=ell, sharpness=8.0), 5)
    m = O.mesh_from_grid(g["occ"], g["labels"])
    vis = O.mesh_vertex_visible(m["edge_ids"], g["labels"])
    z = m["verts"][:, 2]
    assert not np.any(vis[z < -0.15])
    # a vertex on a z edge is visible exactly when it is its column's first crossing seen
    # from z = +1 (a scan down the column)
    lab = g["labels"]
    n = lab.shape[0]
    zedge = (m["edge_ids"] % 3) == 2
    for g_id, v in zip(m["edge_ids"][zedge], vis[zedge]):
        node = int(g_id // 3)
        i, j, k = node // (n * n), (node // n) % n, node % n
        first = next(kk for kk in range(n - 2, -1, -1) if lab[i, j, kk] != lab[i, j, kk + 1])
        assert v == (k == first), (i, j, k, first)
    assert np.all(vis[zedge & (z > 0.15)])


def test_colors_take_the_pixel_where_visible():
    feat = synth.feature_map(32, 32, 64, 4.0, 5)
    spec = synth.he_mlp(64, 2, [64, 3], [False] * 2, 6, hidden_act="lrelu", out_act="tanh")
    col = O.Field("mlp", feat=feat, mlp=spec)
    img = np.tanh(synth.feature_map(64, 64, 3, 6.0, 9))
    verts = np.array([[0.1, 0.2, 0.3], [-0.5, 0.4, -0.2]])
    c = O.mesh_colors(verts, np.array([True, False]), img, col)
    assert np.allclose(c[0], O.bilinear_sample(img, verts[:1, 0], verts[:1, 1])[0], atol=0)
    f = O.bilinear_sample(feat, verts[1:, 0], verts[1:, 1])
    want = np.tanh(O.mlp_preact(spec, f, np.array([[-0.2, 0.5]])))
    assert np.allclose(c[1], want[0], atol=0)
