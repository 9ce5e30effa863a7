"""Exact render parity where the full-size code paths run.

The ray kernels keep a coarse column's labels as 64-node bit masks; at the benchmarked
depth (512 x 512 x 256 from 64 x 64 x 32) a level-(L-1) column holds 129 nodes, three
words, so the cross-word shifts of the mask walk are in play.  These tests compare the
traced render (k*, k1, the evaluation level and logit of every node) with the oracle
element by element:
  * at 256 x 256 x 256 from 32^3 (129 nodes per coarse column) on the tiny MLP and on an
    ellipsoid union, yaw 0, 90 and 180: against the oracle's own render;
  * at the benchmarked 512 x 512 x 256 with the PIFu-size network: the oracle's render
    replayed on the GPU's recorded logits must request exactly the nodes the GPU
    evaluated at every level and reproduce k*, k1, hits, depth and stats; sampled
    evaluated nodes and hit colours are checked against the oracle's network.
"""
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


def _oracle_eval_map(r, lw, ld):
    """Level at which the oracle's render evaluated each node of the finest lattice."""
    W, D = 1 << lw, 1 << ld
    out = np.full((W + 1, W + 1, D + 1), 255, np.uint8)
    T = len(r["levels"])
    for t, rec in enumerate(r["levels"]):
        s = 1 << (T - t)
        m = np.zeros(int(np.prod(rec.dims)), bool)
        m[rec.evaluated] = True
        sub = out[::s, ::s, ::s]
        sub[m.reshape(rec.dims)] = rec.level
    idx = r["last_eval"]
    ii, jj, kk = idx // (W * (D + 1)), (idx // (D + 1)) % W, idx % (D + 1)
    out[ii, jj, kk] = lw
    return out


def _compare(gpu, ref, lw, ld, rgb_tol=1e-4, depth_tol=1e-4):
    hit = gpu["hit"].cpu().numpy()
    assert np.array_equal(hit, ref["hit"]), "hits differ"
    assert np.array_equal(gpu["kstar"].cpu().numpy(), ref["kstar"]), "k* differs"
    assert np.array_equal(gpu["k1"].cpu().numpy(), ref["k1"]), "k1 differs"
    d = gpu["depth"].cpu().numpy()
    assert np.array_equal(np.isnan(d), np.isnan(ref["depth"]))
    if hit.any():
        assert np.max(np.abs(d[hit == 1] - ref["depth"][hit == 1])) <= depth_tol
    if ref["rgb"] is not None:
        assert np.max(np.abs(gpu["rgb"].cpu().numpy() - ref["rgb"])) <= rgb_tol
    evl = gpu["eval_level"].cpu().numpy()
    assert np.array_equal(evl, _oracle_eval_map(ref, lw, ld)), "evaluated sets differ"
    for g, rec in zip(gpu["stats"][:-1], ref["levels"]):
        for k in ("nodes", "b0", "dilated", "evaluated", "waves", "conflicts"):
            assert g[k] == rec.stats[k], (rec.level, k, g[k], rec.stats[k])
    last = gpu["stats"][-1]
    assert last["evaluated"] == ref["stats"]["evaluated_last"]
    assert last["shadow"] == ref["stats"]["shadow"]
    assert last["hits"] == ref["stats"]["hits"]


def _color(C=64, seed=5):
    feat = synth.feature_map(32, 32, C, 4.0, seed)
    spec = synth.he_mlp(C, 2, [128, 64, 3], [False, False, False], seed + 1, hidden_act="lrelu",
                        out_act="tanh")
    return feat, spec


@pytest.mark.parametrize("yaw", [0.0, 90.0, 180.0])
@pytest.mark.parametrize("kind", ["mlp", "ell"])
def test_render_three_word_columns_exact(pifu, kind, yaw):
    lw, ld, lc = 8, 8, 5
    if kind == "mlp":
        feat, spec = synth.tiny_features(), synth.tiny_mlp()
        fo = O.Field("mlp", feat=feat, mlp=spec)
        fg = pifu.DeviceField.mlp_field(feat, spec)
    else:
        ell = synth.ellipsoids(8, 302)
        fo = O.Field("ellipsoids", ell=ell, sharpness=8.0)
        fg = pifu.DeviceField.ellipsoids(ell, 8.0)
    cfeat, cspec = _color()
    co = O.Field("mlp", feat=cfeat, mlp=cspec)
    cg = pifu.DeviceField.mlp_field(cfeat, cspec)
    view = synth.yaw_view(yaw)
    bg = (0.2, 0.4, 0.6)
    gpu = pifu.render_view_traced(fg, cg, view, lw, ld, lc, bg)
    torch.cuda.synchronize()
    print(f"[render exact] kind={kind} yaw={yaw} sizes=({lw},{ld},{lc})", flush=True)
    ref = O.render_view(fo, co, view, lw, ld, lc, bg)
    assert (1 << (ld - 1)) + 1 > 128          # level L-1 columns span three 64-node words
    assert ref["hit"].sum() > 1000
    _compare(gpu, ref, lw, ld)
    # evaluated nodes: the network's logit against the oracle's
    evl = gpu["eval_level"].cpu().numpy()
    lg = gpu["logit"].cpu().numpy()
    ii, jj, kk = np.nonzero(evl != 255)
    sel = np.random.default_rng(1).choice(ii.size, min(4000, ii.size), replace=False)
    W, D = 1 << lw, 1 << ld
    P = np.stack([-1 + 2.0 * ii[sel] / W, -1 + 2.0 * jj[sel] / W, -1 + 2.0 * kk[sel] / D], 1)
    ref_lg = O.view_logit(fo, view, P)
    got = lg[ii[sel], jj[sel], kk[sel]].astype(np.float64)
    fin = np.isfinite(ref_lg)
    assert np.array_equal(got[fin] > 0, ref_lg[fin] > 0)
    assert np.all(got[~fin] < -1e30)
    assert np.max(np.abs(O.sigmoid(got[fin]) - O.sigmoid(ref_lg[fin]))) <= 1e-4


def test_render_full_size_replay(pifu):
    """512 x 512 x 256 from 64 x 64 x 32 with the PIFu-size networks at yaw 90 (the
    benchmarked render): exact replay of every level, then sampled values."""
    lw, ld, lc = 9, 8, 6
    W, D = 1 << lw, 1 << ld
    feat, spec = synth.pifu_features(), synth.pifu_mlp()
    fg = pifu.DeviceField.mlp_field(feat, spec)
    cfeat, cspec = synth.color_features(), synth.color_mlp()
    cg = pifu.DeviceField.mlp_field(cfeat, cspec)
    view = synth.yaw_view(90.0)
    gpu = pifu.render_view_traced(fg, cg, view, lw, ld, lc)
    torch.cuda.synchronize()
    print("[render replay] 512x512x256 yaw 90 traced", flush=True)
    evl = gpu["eval_level"].cpu().numpy()
    lg = gpu["logit"].cpu().numpy()

    def lookup(P):
        i = np.rint((P[:, 0] + 1.0) * 0.5 * W).astype(np.int64)
        j = np.rint((P[:, 1] + 1.0) * 0.5 * W).astype(np.int64)
        k = np.rint((P[:, 2] + 1.0) * 0.5 * D).astype(np.int64)
        assert np.all(evl[i, j, k] != 255), "the oracle asked for a node the GPU never evaluated"
        return lg[i, j, k].astype(np.float64)

    ref = O.render_view(None, None, view, lw, ld, lc, evaluate=lookup)
    ref["rgb"] = None
    print(f"[render replay] hits {int(ref['hit'].sum())}", flush=True)
    _compare(gpu, ref, lw, ld, depth_tol=1e-5)
    # the recorded logits against the oracle's network on sampled evaluated nodes
    fo = O.Field("mlp", feat=feat, mlp=spec)
    ii, jj, kk = np.nonzero(evl != 255)
    sel = np.random.default_rng(2).choice(ii.size, 3000, replace=False)
    P = np.stack([-1 + 2.0 * ii[sel] / W, -1 + 2.0 * jj[sel] / W, -1 + 2.0 * kk[sel] / D], 1)
    ref_lg = O.view_logit(fo, view, P)
    got = lg[ii[sel], jj[sel], kk[sel]].astype(np.float64)
    fin = np.isfinite(ref_lg)
    assert np.array_equal(got[fin] > 0, ref_lg[fin] > 0)
    assert np.all(got[~fin] < -1e30)
    assert np.max(np.abs(O.sigmoid(got[fin]) - O.sigmoid(ref_lg[fin]))) <= 1e-4
    # colours of sampled hits: the oracle's colour network at the GPU's hit point, with the
    # occupancy input the replay assigns to node k1
    hit = gpu["hit"].cpu().numpy()
    vs, us = np.nonzero(hit)
    s = np.random.default_rng(3).choice(us.size, min(2000, us.size), replace=False)
    u, v = us[s], vs[s]
    z = gpu["depth"].cpu().numpy()[v, u].astype(np.float64)
    k1 = gpu["k1"].cpu().numpy()[v, u]
    x, y = -1.0 + 2.0 * u / W, -1.0 + 2.0 * v / W
    evk = evl[u, v, k1] != 255
    occ = np.where(evk, O.sigmoid(lg[u, v, k1].astype(np.float64)), 1.0)
    Pp, _ = O.apply_view(view, np.stack([x, y, z], 1))
    f = O.bilinear_sample(cfeat, Pp[:, 0], Pp[:, 1])
    rgb_ref = np.tanh(O.mlp_preact(cspec, f, np.stack([Pp[:, 2], occ], 1)))
    assert np.max(np.abs(gpu["rgb"].cpu().numpy()[v, u] - rgb_ref)) <= 1e-4
