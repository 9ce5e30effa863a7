"""GPU training kernels (through the C ABI) against the FP64 oracle: BCE gradient,
backward pass, RMSProp, determinism, and a loss that goes down."""
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


def _batch(C, n, seed, feat_hw=32):
    feat = synth.feature_map(feat_hw, feat_hw, C, 4.0, seed)
    g = np.random.default_rng(seed)
    pts = np.zeros((n, 4), np.float32)
    pts[:, :3] = g.uniform(-1, 1, (n, 3))
    pts[:, 3] = g.uniform(0, 1, n)
    return feat, pts


@pytest.mark.parametrize("which", ["plain", "skip", "surrogate"])
def test_mlp_grad_matches_oracle(pifu, which):
    from paper_2007_13988_amd.train import MLPTrainer
    if which == "plain":
        spec = synth.he_mlp(64, 1, [64, 64, 1], [False, False, False], 41)
        C = 64
    elif which == "skip":
        spec = synth.he_mlp(64, 1, [128, 64, 1], [False, True, False], 42)
        C = 64
    else:
        spec = synth.surrogate_mlp()
        C = 256
    feat, pts = _batch(C, 3000, 43)
    net = pifu.DeviceMLP(spec)
    tr = MLPTrainer(net, 4096)
    loss = tr.grad(torch.from_numpy(feat).cuda(), torch.from_numpy(pts).cuda())
    torch.cuda.synchronize()
    P64 = pts[:, :3].astype(np.float64)
    f = O.bilinear_sample(feat, P64[:, 0], P64[:, 1])
    ins, pres = O.mlp_forward_cache(spec, f, P64[:, 2:3])
    ref_loss, ds = O.bce_soft(pres[-1][:, 0], pts[:, 3].astype(np.float64))
    dW, db = O.mlp_backward(spec, ins, pres, ds[:, None])
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * max(1.0, abs(ref_loss))
    for l in range(len(spec.widths)):
        gw = tr.dW[l].cpu().numpy().astype(np.float64)
        gb = tr.db[l].cpu().numpy().astype(np.float64)
        scale_w = np.max(np.abs(dW[l])) + 1e-12
        scale_b = np.max(np.abs(db[l])) + 1e-12
        assert np.max(np.abs(gw - dW[l])) <= 1e-4 * scale_w, (l, np.max(np.abs(gw - dW[l])), scale_w)
        assert np.max(np.abs(gb - db[l])) <= 1e-4 * scale_b, (l, np.max(np.abs(gb - db[l])), scale_b)


def test_grad_is_bit_reproducible(pifu):
    from paper_2007_13988_amd.train import MLPTrainer
    spec = synth.surrogate_mlp()
    feat, pts = _batch(256, 20000, 44)
    net = pifu.DeviceMLP(spec)
    tr = MLPTrainer(net, 20000)
    ft, pt = torch.from_numpy(feat).cuda(), torch.from_numpy(pts).cuda()
    tr.grad(ft, pt)
    first = [t.clone() for t in tr.dW + tr.db]
    tr.grad(ft, pt)
    for a, b in zip(first, tr.dW + tr.db):
        assert torch.equal(a, b)


def test_rmsprop_step_matches_oracle(pifu):
    from paper_2007_13988_amd.train import MLPTrainer
    spec = synth.he_mlp(64, 1, [64, 64, 1], [False, False, False], 45)
    feat, pts = _batch(64, 2000, 46)
    net = pifu.DeviceMLP(spec)
    tr = MLPTrainer(net, 2000)
    ft, pt = torch.from_numpy(feat).cuda(), torch.from_numpy(pts).cuda()
    W0 = [w.cpu().numpy().astype(np.float64) for w in net.W]
    v = [np.zeros_like(w) for w in W0]
    for step in range(3):
        tr.grad(ft, pt)
        g = [d.cpu().numpy().astype(np.float64) for d in tr.dW]
        tr.step()
        for l in range(3):
            W0[l], v[l] = O.rmsprop_step(W0[l], g[l], v[l])
    for l in range(3):
        assert np.max(np.abs(net.W[l].cpu().numpy() - W0[l])) <= 1e-6


def test_checkpoint_resume_is_bit_exact(pifu, tmp_path):
    """Stopping after k steps, checkpointing, and resuming in a fresh trainer gives the
    same weights as training straight through (deterministic kernels)."""
    from paper_2007_13988_amd.train import MLPTrainer
    spec = synth.surrogate_mlp(77)
    feat, pts = _batch(256, 8192, 49)
    ft, pt = torch.from_numpy(feat).cuda(), torch.from_numpy(pts).cuda()
    a = MLPTrainer(pifu.DeviceMLP(spec), 8192)
    for _ in range(6):
        a.grad(ft, pt)
        a.step()
    b = MLPTrainer(pifu.DeviceMLP(spec), 8192)
    for _ in range(3):
        b.grad(ft, pt)
        b.step()
    ck = str(tmp_path / "ck.npz")
    b.save(ck, step=3)
    c = MLPTrainer(pifu.DeviceMLP(synth.surrogate_mlp(78)), 8192)
    assert c.load(ck) == 3
    for _ in range(3):
        c.grad(ft, pt)
        c.step()
    for wa, wc in zip(a.net.W + a.net.b, c.net.W + c.net.b):
        assert torch.equal(wa, wc)


def test_training_lowers_the_distillation_loss(pifu):
    from paper_2007_13988_amd.train import MLPTrainer
    teacher = synth.tiny_mlp()
    feat = synth.tiny_features()
    fo = O.Field("mlp", feat=feat, mlp=teacher)
    g = np.random.default_rng(47)
    pts = np.zeros((16384, 4), np.float32)
    pts[:, :3] = g.uniform(-1, 1, (16384, 3))
    pts[:, 3] = O.sigmoid(O.field_logit(fo, pts[:, :3].astype(np.float64)))
    student = synth.he_mlp(64, 1, [64, 64, 1], [False, False, False], 48)
    net = pifu.DeviceMLP(student)
    tr = MLPTrainer(net, 16384, lr=3e-3)
    ft, pt = torch.from_numpy(feat).cuda(), torch.from_numpy(pts).cuda()
    first = float(tr.grad(ft, pt).item())
    for _ in range(200):
        tr.grad(ft, pt)
        tr.step()
    last = float(tr.grad(ft, pt).item())
    t = pts[:, 3].astype(np.float64).clip(1e-12, 1 - 1e-12)
    entropy = float(np.mean(-t * np.log(t) - (1 - t) * np.log(1 - t)))   # the loss floor
    assert last - entropy < 0.5 * (first - entropy), (first, last, entropy)
