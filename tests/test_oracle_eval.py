"""Pins of the oracle's point evaluation: bilinear sampling, MLP wiring, FLOP counts,
number formats and training maths, each against an independent routine."""
import json
import math
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as Fnn

import synth
from oracle import pifu_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_bilinear_matches_grid_sample_fp64_zero_padding():
    g = np.random.default_rng(1)
    F = g.standard_normal((7, 9, 5))
    xy = g.uniform(-1.3, 1.3, (400, 2))
    xy[:8] = [[-1, -1], [1, 1], [-1, 1], [1, -1], [0, 0], [1, 0.3], [-0.2, 1], [1.0, 1.2]]
    got = O.bilinear_sample(F, xy[:, 0], xy[:, 1])
    inp = torch.from_numpy(np.transpose(F, (2, 0, 1))[None].copy())
    grid = torch.from_numpy(xy[None, None].copy())
    ref = Fnn.grid_sample(inp, grid, mode="bilinear", padding_mode="zeros", align_corners=True)
    ref = ref[0, :, 0, :].T.numpy()
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def test_bilinear_exact_on_affine_feature_maps():
    H, W, C = 9, 13, 3
    a = np.array([1.0, -2.0, 0.5])
    b = np.array([3.0, 0.25, -1.0])
    d = np.array([0.5, 1.0, 2.0])
    vv, uu = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    F = uu[..., None] * a + vv[..., None] * b + d
    g = np.random.default_rng(2)
    x = g.uniform(-1, 1, 200)
    y = g.uniform(-1, 1, 200)
    u = (x + 1) / 2 * (W - 1)
    v = (y + 1) / 2 * (H - 1)
    expect = u[:, None] * a + v[:, None] * b + d
    assert np.allclose(O.bilinear_sample(F, x, y), expect, rtol=0, atol=1e-12)


class _TorchMLP(torch.nn.Module):
    """Independent torch construction of the skip-concat MLP (fp64)."""

    def __init__(self, spec):
        super().__init__()
        self.spec = spec
        self.lin = torch.nn.ModuleList()
        for l, n_out in enumerate(spec.widths):
            lin = torch.nn.Linear(spec.in_width(l), n_out).double()
            with torch.no_grad():
                lin.weight.copy_(torch.from_numpy(spec.W[l].astype(np.float64)))
                lin.bias.copy_(torch.from_numpy(spec.b[l].astype(np.float64)))
            self.lin.append(lin)

    def forward(self, f, extras):
        h = torch.cat([f, extras], dim=1)
        for l, lin in enumerate(self.lin):
            if l > 0 and self.spec.skip[l]:
                h = torch.cat([h, f], dim=1)
            h = lin(h)
            if l < len(self.lin) - 1:
                h = torch.relu(h) if self.spec.hidden_act == "relu" else Fnn.leaky_relu(h, 0.01)
        return h


@pytest.mark.parametrize("which", ["tiny", "pifu", "color", "surrogate"])
def test_mlp_matches_torch_modules(which):
    spec = {"tiny": synth.tiny_mlp, "pifu": synth.pifu_mlp, "color": synth.color_mlp,
            "surrogate": synth.surrogate_mlp}[which]()
    g = np.random.default_rng(3)
    f = g.standard_normal((64, spec.feat_dim))
    ex = g.uniform(-1, 1, (64, spec.n_extra))
    got = O.mlp_preact(spec, f, ex)
    ref = _TorchMLP(spec)(torch.from_numpy(f), torch.from_numpy(ex)).detach().numpy()
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_pifu_mlp_cost_matches_paper_table2():
    """Tab. 2 lists 9.7 GFLOPs per 4096 calls for the PIFu MLP (two significant figures)."""
    ref = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    spec = synth.pifu_mlp()
    per_point = spec.flops_per_point()
    assert per_point == 2_361_600
    assert spec.n_params() == 1_182_721
    table = ref["tab2_mlp_gflops_per_4096_calls"]["value"]
    assert round(per_point * 4096 / 1e9, 1) == table


def test_field_mlp_is_bilinear_then_mlp():
    feat = synth.tiny_features()
    spec = synth.tiny_mlp()
    fld = O.Field("mlp", feat=feat, mlp=spec)
    P = np.random.default_rng(4).uniform(-1, 1, (50, 3))
    f = O.bilinear_sample(feat, P[:, 0], P[:, 1])
    ref = _TorchMLP(spec)(torch.from_numpy(f), torch.from_numpy(P[:, 2:3].copy())).detach().numpy()
    assert np.allclose(O.field_logit(fld, P), ref[:, 0], rtol=1e-12, atol=1e-12)


def test_view_transform_and_clip():
    v = synth.yaw_view(90.0)
    P = np.array([[0.5, 0.1, -0.3], [1.0, 0.0, 1.0], [0.2, 0.2, 0.9]])
    Pp, inside = O.apply_view(v, P)
    # yaw 90 deg: x' = z, y' = y, z' = -x
    assert np.allclose(Pp, np.stack([P[:, 2], P[:, 1], -P[:, 0]], axis=1), atol=1e-7)
    assert inside.all()
    v45 = synth.yaw_view(45.0)
    _, ins = O.apply_view(v45, np.array([[0.9, 0, 0.9], [0.1, 0, 0.1]]))
    assert list(ins) == [False, True]
    fld = O.Field("plane", plane=np.array([0, 0, 0, 1.0]))
    lg = O.view_logit(fld, v45, np.array([[0.9, 0, 0.9], [0.1, 0, 0.1]]))
    assert lg[0] == -np.inf and lg[1] == 1.0


# ---------------------------------------------------------------- number formats

def test_bf16_rounding_matches_torch_cast():
    g = np.random.default_rng(6)
    x = np.concatenate([g.standard_normal(10000).astype(np.float32) * 10,
                        np.array([0.0, -0.0, 1.0, 3.0e38, 1e-40, -2.5], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(O.to_bf16(x), ref)


def test_e4m3_rounding_matches_torch_cast_in_range():
    g = np.random.default_rng(7)
    x = np.concatenate([g.standard_normal(20000) * 40, g.uniform(-448, 448, 2000),
                        np.ldexp(1.0, np.arange(-12, 9)), [0.0, 2.0 ** -10, 3 * 2.0 ** -10]])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    assert np.array_equal(O.to_e4m3(x), ref)


def test_e4m3_saturates():
    assert O.to_e4m3(np.array([1000.0, -1e6, 449.0, 464.0]))[0] == 448.0
    assert list(O.to_e4m3(np.array([1000.0, -1e6, 449.0, 464.0]))) == [448.0, -448.0, 448.0, 448.0]
    # the largest finite values and the spacing near them (exponent 8: step 32)
    assert list(O.to_e4m3(np.array([416.0, 432.0, 431.0]))) == [416.0, 448.0, 416.0]


# ---------------------------------------------------------------- training maths

def test_bce_soft_matches_torch_and_finite_differences():
    g = np.random.default_rng(8)
    s = g.standard_normal(50) * 3
    t = g.uniform(0, 1, 50)
    loss, grad = O.bce_soft(s, t)
    ref = Fnn.binary_cross_entropy_with_logits(torch.from_numpy(s), torch.from_numpy(t))
    assert abs(loss - ref.item()) < 1e-12
    h = 1e-6
    for i in range(5):
        e = np.zeros_like(s)
        e[i] = h
        fd = (O.bce_soft(s + e, t)[0] - O.bce_soft(s - e, t)[0]) / (2 * h)
        assert abs(fd - grad[i]) < 1e-8


@pytest.mark.parametrize("act", ["relu", "lrelu"])
def test_mlp_backward_matches_autograd_and_finite_differences(act):
    spec = synth.he_mlp(6, 1, [8, 5, 1], [False, True, False], 31, hidden_act=act)
    g = np.random.default_rng(9)
    f = g.standard_normal((20, 6))
    z = g.uniform(-1, 1, (20, 1))
    tgt = g.uniform(0, 1, 20)
    ins, pres = O.mlp_forward_cache(spec, f, z)
    loss, ds = O.bce_soft(pres[-1][:, 0], tgt)
    dW, db = O.mlp_backward(spec, ins, pres, ds[:, None])
    m = _TorchMLP(spec)
    out = m(torch.from_numpy(f), torch.from_numpy(z))[:, 0]
    Fnn.binary_cross_entropy_with_logits(out, torch.from_numpy(tgt)).backward()
    for l, lin in enumerate(m.lin):
        assert np.allclose(dW[l], lin.weight.grad.numpy(), rtol=1e-10, atol=1e-12)
        assert np.allclose(db[l], lin.bias.grad.numpy(), rtol=1e-10, atol=1e-12)
    # central differences on a few weights of every layer
    h = 1e-6
    for l in range(3):
        W0 = spec.W[l].astype(np.float64)
        for (a, b) in [(0, 0), (W0.shape[0] - 1, 2)]:
            spec.W[l] = W0.copy()
            spec.W[l][a, b] += h
            lp = O.bce_soft(O.mlp_preact(spec, f, z)[:, 0], tgt)[0]
            spec.W[l] = W0.copy()
            spec.W[l][a, b] -= h
            lm = O.bce_soft(O.mlp_preact(spec, f, z)[:, 0], tgt)[0]
            spec.W[l] = W0
            assert abs((lp - lm) / (2 * h) - dW[l][a, b]) < 1e-7


def test_rmsprop_matches_torch_optimizer():
    g = np.random.default_rng(10)
    w = g.standard_normal(30)
    v = np.zeros(30)
    p = torch.nn.Parameter(torch.from_numpy(w.copy()))
    opt = torch.optim.RMSprop([p], lr=1e-3, alpha=0.99, eps=1e-8)
    for step in range(5):
        grad = g.standard_normal(30)
        w, v = O.rmsprop_step(w, grad, v)
        p.grad = torch.from_numpy(grad.copy())
        opt.step()
    assert np.allclose(w, p.detach().numpy(), rtol=0, atol=1e-14)
