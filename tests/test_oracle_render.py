"""Pins of the oracle's mesh-free renderer (Sec. 3.2 and Eq. 3).

Checks: a per-ray brute force written with plain loops, the closed-form depth of
a sphere, rotation invariance for a centred sphere, exact background pixels and
agreement of the hit index with a ray search over dense labels.
"""
import itertools
import math

import numpy as np
import pytest
import torch

import synth
from brute import brute_localize
from oracle import pifu_oracle as O


def _sphere(r=0.6):
    return O.Field("ellipsoids", ell=synth.sphere_as_ellipsoid(r), sharpness=8.0)


def _color_field(C=8, seed=5):
    feat = synth.feature_map(16, 16, C, 2.0, seed)
    mlp = synth.he_mlp(C, 2, [16, 8, 3], [False, False, False], seed + 1,
                       hidden_act="lrelu", out_act="tanh")
    return O.Field("mlp", feat=feat, mlp=mlp)


def _brute_render(occ_fld, col_fld, view, lw, ld, lcw, bg):
    """Per-ray brute force of the last render level (plain loops)."""
    T = lw - lcw
    W, D = 1 << lw, 1 << ld
    # levels below L: the plain-loop closure on the anisotropic target lattice
    fn = lambda P: float(O.view_logit(occ_fld, view, np.array([P]))[0])
    _, labc, _, valc, _ = brute_localize(fn, (1 << (lw - T), 1 << (lw - T), 1 << (ld - T)), T - 1, 7)
    V = np.asarray(view, np.float64).reshape(3, 4)
    rgb = np.zeros((W, W, 3)) + np.asarray(bg)
    depth = np.full((W, W), np.nan)
    hit = np.zeros((W, W), np.uint8)
    n_eval = 0
    for u in range(W):
        for v in range(W):
            vals = {}
            labs = {}
            interp = {}
            for k in range(D + 1):
                cs = list(itertools.product(sorted({u // 2, (u + 1) // 2}), sorted({v // 2, (v + 1) // 2}),
                                            sorted({k // 2, (k + 1) // 2})))
                interp[k] = sum(int(labc[c]) for c in cs) / len(cs)
            kstar = None
            for k in range(D, -1, -1):
                if interp[k] == 1.0:
                    kstar = k
                    break
            for k in range(D + 1):
                coarse = u % 2 == 0 and v % 2 == 0 and k % 2 == 0
                if coarse:
                    c = (u // 2, v // 2, k // 2)
                    vals[k] = valc[c]
                    labs[k] = int(labc[c])
                    continue
                shadow = kstar is not None and k < kstar
                if not shadow and 0 < interp[k] < 1:
                    P = np.array([[-1 + 2 * u / W, -1 + 2 * v / W, -1 + 2 * k / D]])
                    lg = O.view_logit(occ_fld, view, P)[0]
                    n_eval += 1
                    vals[k] = 1 / (1 + math.exp(-lg)) if lg > -np.inf else 0.0
                    labs[k] = int(lg > 0)
                else:
                    vals[k] = interp[k]
                    labs[k] = int(interp[k] == 1.0)
            k1 = None
            for k in range(D, -1, -1):
                if labs[k] == 1:
                    k1 = k
                    break
            if k1 is None:
                continue
            if k1 == D:
                z = 1.0
            else:
                of, ob = vals[k1 + 1], vals[k1]
                t = (0.5 - of) / (ob - of) if ob > of else 0.0
                z = (-1 + 2 * (k1 + 1) / D) + t * (2 * k1 / D - 2 * (k1 + 1) / D)
            depth[u, v] = z
            hit[u, v] = 1
            P = V[:, :3] @ np.array([-1 + 2 * u / W, -1 + 2 * v / W, z]) + V[:, 3]
            f = O.bilinear_sample(col_fld.feat, np.array([P[0]]), np.array([P[1]]))
            ft = torch.from_numpy(f)
            h = torch.cat([ft, torch.tensor([[P[2], vals[k1]]], dtype=torch.float64)], 1)
            spec = col_fld.mlp
            for l in range(len(spec.widths)):
                h = h @ torch.from_numpy(spec.W[l].astype(np.float64)).T + torch.from_numpy(
                    spec.b[l].astype(np.float64))
                if l < len(spec.widths) - 1:
                    h = torch.nn.functional.leaky_relu(h, 0.01)
            rgb[u, v] = torch.tanh(h)[0].numpy()
    return rgb.transpose(1, 0, 2), depth.T, hit.T, n_eval


@pytest.mark.parametrize("yaw,kind,sizes", [(0.0, "mlp", (4, 3, 2)), (45.0, "mlp", (4, 3, 2)),
                                            (45.0, "ell", (5, 4, 3)), (180.0, "ell", (5, 4, 3)),
                                            (90.0, "mlp", (4, 4, 2))])
def test_render_matches_per_ray_brute_force(yaw, kind, sizes):
    if kind == "mlp":
        feat = synth.feature_map(16, 16, 8, 2.0, 3)
        occ = O.Field("mlp", feat=feat, mlp=synth.he_mlp(8, 1, [16, 8, 1], [False] * 3, 4))
    else:
        occ = O.Field("ellipsoids", ell=synth.ellipsoids(4, 12), sharpness=8.0)
    col = _color_field()
    view = synth.yaw_view(yaw)
    bg = (0.25, -0.5, 1.0)
    r = O.render_view(occ, col, view, *sizes, bg)
    rgb, depth, hit, n_eval = _brute_render(occ, col, view, *sizes, bg)
    assert hit.sum() > 0
    assert np.array_equal(r["hit"], hit)
    assert np.array_equal(np.isnan(r["depth"]), np.isnan(depth))
    assert np.allclose(r["depth"][hit == 1], depth[hit == 1], rtol=0, atol=1e-12)
    assert np.allclose(r["rgb"], rgb, rtol=0, atol=1e-12)
    assert r["stats"]["evaluated_last"] == n_eval


def test_sphere_depth_closed_form_and_background():
    rad = 0.6
    lw, ld = 5, 5
    r = O.render_view(_sphere(rad), _color_field(), synth.yaw_view(0.0), lw, ld, 3, (0.1, 0.2, 0.3))
    W, D = 1 << lw, 1 << ld
    v, u = np.meshgrid(np.arange(W), np.arange(W), indexing="ij")
    x = -1 + 2 * u / W
    y = -1 + 2 * v / W
    rr = x * x + y * y
    inner = rr < (rad - 2.0 / W) ** 2
    outer = rr > (rad + 2.0 / W) ** 2
    assert r["hit"][inner].all()
    assert not r["hit"][outer].any()
    zt = np.sqrt(rad * rad - rr[inner])
    assert np.max(np.abs(r["depth"][inner] - zt)) <= 2.0 / D
    bgpix = r["hit"] == 0
    assert np.all(r["rgb"][bgpix] == np.array([0.1, 0.2, 0.3]))
    assert np.all(np.isnan(r["depth"][bgpix]))


def test_identity_view_hit_index_matches_dense_ray_search():
    rad = 0.6
    lw = ld = 5
    r = O.render_view(_sphere(rad), _color_field(), synth.yaw_view(0.0), lw, ld, 3)
    d = O.dense_grid(_sphere(rad), 5)["labels"]       # [i=x, j=y, k=z]
    W = 1 << lw
    kk = np.arange(d.shape[2])
    k_dense = np.where(d.any(axis=2), np.max(np.where(d == 1, kk, -1), axis=2), -1)[:W, :W].T
    assert np.array_equal(r["k1"], k_dense)


@pytest.mark.parametrize("yaw", [90.0, 180.0, 270.0])
def test_centred_sphere_render_is_rotation_invariant(yaw):
    a = O.render_view(_sphere(), _color_field(), synth.yaw_view(0.0), 5, 4, 3)
    b = O.render_view(_sphere(), _color_field(), synth.yaw_view(yaw), 5, 4, 3)
    assert np.array_equal(a["hit"], b["hit"])
    assert np.allclose(a["depth"][a["hit"] == 1], b["depth"][b["hit"] == 1], atol=1e-12)


def test_no_shadow_node_is_evaluated():
    feat = synth.feature_map(16, 16, 8, 2.0, 3)
    occ = O.Field("mlp", feat=feat, mlp=synth.he_mlp(8, 1, [16, 8, 1], [False] * 3, 4, out_bias=1.0))
    r = O.render_view(occ, _color_field(), synth.yaw_view(0.0), 5, 4, 3)
    kk = np.arange(r["eval_mask_last"].shape[2])
    kstar = r["kstar"].T
    shadow = kk[None, None, :] < kstar[:, :, None]
    assert not (shadow & r["eval_mask_last"]).any()
    assert r["stats"]["shadow"] > 0
