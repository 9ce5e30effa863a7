"""Pins of the oracle's CBN + SoftZ lifting network (appendix, "Depth Representation",
"Pixel-aligned 3D Lifting"; Tab. 2): the soft one-hot code against its closed forms,
batch norm against torch's inference-mode batch_norm, the whole network against an
independent torch composition, and its FLOP count against Tab. 2."""
import json
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

import synth
from oracle import pifu_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_softz_closed_forms():
    n = 64
    z = np.linspace(-1, 1, 1001)
    Z = O.softz(z, n)
    assert np.all(Z >= 0) and np.allclose(Z.sum(1), 1.0, atol=1e-15)
    assert np.all((Z > 0).sum(1) <= 2)
    # linear interpolation of the bin positions reproduces P'_z
    assert np.allclose(Z @ (np.arange(n) / (n - 1)), 0.5 * (z + 1), atol=1e-14)
    # the ends and the bin centres are one-hot
    assert Z[0, 0] == 1.0 and Z[-1, n - 1] == 1.0
    zc = 2.0 * np.arange(n) / (n - 1) - 1.0
    assert np.allclose(O.softz(zc, n), np.eye(n), atol=1e-12)
    # depths outside [-1, 1] take the code of the nearest end
    assert np.array_equal(O.softz(np.array([-1.5, 1.25]), n), O.softz(np.array([-1.0, 1.0]), n))


def test_conditional_batch_norm_against_torch():
    net = synth.cbn_net(feat_dim=16, n_z=8, width=32, n_blocks=1, seed=3)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((50, 16))
    z = rng.uniform(-1, 1, 50)
    h = O.softz(z, 8) @ net.Wp.astype(np.float64).T + net.bp
    bn = Fn.batch_norm(torch.from_numpy(h), torch.from_numpy(net.mean[0].astype(np.float64)),
                       torch.from_numpy(net.var[0].astype(np.float64)), training=False,
                       eps=net.eps).numpy()
    gamma = f @ net.Wg[0].astype(np.float64).T + net.bg[0]
    beta = f @ net.Wb[0].astype(np.float64).T + net.bb[0]
    a = np.maximum(gamma * bn + beta, 0)
    want = a @ net.Wo.astype(np.float64).T + net.bo
    assert np.allclose(O.cbn_logit(net, f, z), want[:, 0], rtol=0, atol=1e-12)


def test_network_against_an_independent_torch_composition():
    net = synth.cbn_net(seed=5)
    rng = np.random.default_rng(1)
    f = torch.from_numpy(rng.standard_normal((200, 256)))
    z = torch.from_numpy(rng.uniform(-1, 1, 200))
    # soft one-hot through torch's one_hot on floor and ceil bins
    s = 63 * 0.5 * (z + 1)
    j = torch.floor(s).long()
    Z = (Fn.one_hot(j.clamp(max=63), 64).double() * (1 + j - s)[:, None] +
         Fn.one_hot((j + 1).clamp(max=63), 64).double() * (s - j)[:, None] * (j + 1 <= 63)[:, None])
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    h = Fn.linear(Z, t(net.Wp), t(net.bp))
    for i in range(net.n_blocks):
        if i:
            h = Fn.linear(a, t(net.W[i - 1]), t(net.b[i - 1]))
        hn = Fn.batch_norm(h, t(net.mean[i]), t(net.var[i]), training=False, eps=net.eps)
        a = torch.relu(Fn.linear(f, t(net.Wg[i]), t(net.bg[i])) * hn + Fn.linear(f, t(net.Wb[i]), t(net.bb[i])))
    want = Fn.linear(a, t(net.Wo), t(net.bo))[:, 0].numpy()
    got = O.cbn_logit(net, f.numpy(), z.numpy())
    assert np.allclose(got, want, rtol=0, atol=1e-10)


def test_flop_count_against_table_2():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    net = synth.cbn_net()
    fl = O.cbn_flops_per_point(net)
    assert fl == 803072
    gf = fl * 4096 / 1e9
    assert abs(gf / g["tab2_cbn_gflops_per_4096_calls"]["value"] - 1) < 0.1, gf


def test_field_has_a_surface():
    """The synthetic CBN field changes sign inside the volume (a surface to localize)."""
    fld = O.Field("cbn", feat=synth.pifu_features(), mlp=synth.cbn_net())
    P = np.random.default_rng(2).uniform(-1, 1, (4000, 3))
    lg = O.field_logit(fld, P)
    frac = float(np.mean(lg > 0))
    assert 0.05 < frac < 0.95, frac


def test_network_carrying_a_closed_form_field():
    """A CBN network built to carry the depth-slab field (synth.depth_slab_cbn with the
    random head term switched off) gives kappa * (tau(c) - |z - mu(c)|) exactly up to
    float32 weights: units 0-3 pass the batch norms unchanged (mean 0, variance 1 - eps)
    and the conditional shifts supply mu and tau.  A dropped term, a wrong sign or a
    transposed map changes the logit by O(1)."""
    import math
    spec = synth.depth_slab_cbn(synth.cbn_net(feat_dim=32, n_z=16, width=64, n_blocks=3,
                                              seed=4, out_bias=0.0), 9, eps=0.0)
    rng = np.random.default_rng(2)
    f = rng.standard_normal((300, 32))
    z = rng.uniform(-1, 1, 300)
    g = synth.rng(9)
    a = g.standard_normal(32)
    a /= np.linalg.norm(a)
    b = g.standard_normal(32)
    b /= np.linalg.norm(b)
    mu = f @ (0.3 * a).astype(np.float32).astype(np.float64)
    tau = f @ (0.25 * b).astype(np.float32).astype(np.float64) + np.float64(np.float32(-0.05))
    want = 16.0 * (tau - np.abs(z - mu))
    bn = 1.0 / math.sqrt(float(np.float32(1.0 - spec.eps)) + spec.eps)   # ~1 + 5e-9
    got = O.cbn_logit(spec, f, z)
    # the bin positions -1 + 2 j / 15 are float32 weights: z is reproduced to ~6e-8
    assert np.max(np.abs(got - want * bn)) <= 2e-6
