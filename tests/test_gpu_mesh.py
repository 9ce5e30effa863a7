"""GPU mesh hand-off (pifu_mesh: Marching Cubes over the surface cells with vertex
colours) against the oracle's mesh of the same grid.

Bar: vertex set (crossed edge ids) and triangles exact -- integer decisions on the labels;
vertex positions within 1e-6 NDC of the oracle's float64 interpolation of the same float32
occupancies; visibility exact; colours within 1e-4 of the oracle's (pixel or colour
network) at the GPU's vertices; and a closed mesh on a closed surface."""
from collections import Counter

import numpy as np
import pytest
import torch

import synth
from oracle import pifu_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pifu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_13988_amd as P
    P.load_library()
    return P


def _color(P):
    feat = synth.feature_map(32, 32, 64, 4.0, 5)
    spec = synth.he_mlp(64, 2, [128, 64, 3], [False] * 3, 6, hidden_act="lrelu", out_act="tanh")
    return P.DeviceField.mlp_field(feat, spec), O.Field("mlp", feat=feat, mlp=spec)


def _check(P, fg, L, l0, with_color=True):
    g = P.occupancy_grid(fg, L, l0)
    cg, co = _color(P)
    img = np.tanh(synth.feature_map(64, 48, 3, 6.0, 9)).astype(np.float32)
    m = P.mesh(g["occ"], g["labels"], g["cells"], cg if with_color else None,
               torch.from_numpy(img).cuda() if with_color else None)
    torch.cuda.synchronize()
    occ = g["occ"].cpu().numpy().astype(np.float64)
    lab = g["labels"].cpu().numpy()
    ref = O.mesh_from_grid(occ, lab)
    print(f"[mesh] 2^{L}: {m['n_verts']} vertices, {m['n_tris']} triangles", flush=True)
    assert m["n_verts"] == ref["verts"].shape[0] and m["n_tris"] == ref["tris"].shape[0]
    assert np.array_equal(m["tris"].cpu().numpy().astype(np.int64), ref["tris"])
    v = m["verts"].cpu().numpy().astype(np.float64)
    assert float(np.max(np.abs(v - ref["verts"]))) <= 1e-6
    if with_color:
        vis = O.mesh_vertex_visible(ref["edge_ids"], lab)
        want = O.mesh_colors(v, vis, img.astype(np.float64), co)
        got = m["colors"].cpu().numpy().astype(np.float64)
        assert float(np.max(np.abs(got - want))) <= 1e-4
        assert 0 < int(vis.sum()) < vis.size
    return m, ref


def test_mesh_of_the_tiny_network(pifu):
    fg = pifu.DeviceField.mlp_field(synth.tiny_features(), synth.tiny_mlp())
    _check(pifu, fg, 5, 3)


def test_mesh_of_ellipsoids_is_closed(pifu):
    fg = pifu.DeviceField.ellipsoids(synth.ellipsoids(8, 302), 8.0)
    m, ref = _check(pifu, fg, 7, 4)
    t = m["tris"].cpu().numpy()
    cnt = Counter((int(a), int(b)) for tri in t for a, b in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0])))
    assert all(c == 1 and (b, a) in cnt for (a, b), c in cnt.items())


def test_mesh_without_colors_and_capacity(pifu):
    fg = pifu.DeviceField.mlp_field(synth.tiny_features(), synth.tiny_mlp())
    g = pifu.occupancy_grid(fg, 5, 3)
    full = pifu.mesh(g["occ"], g["labels"], g["cells"])
    few_t = pifu.mesh(g["occ"], g["labels"], g["cells"], tri_cap=50)
    few_v = pifu.mesh(g["occ"], g["labels"], g["cells"], vert_cap=100)
    torch.cuda.synchronize()
    for cut in (few_t, few_v):
        assert cut["n_verts"] == full["n_verts"] and cut["n_tris"] == full["n_tris"]
    assert torch.equal(few_t["tris"], full["tris"][:50])
    assert torch.equal(few_v["verts"], full["verts"][:100])
