"""Point-OHEM on the GPU (Sec. 3.3, Eq. 6 right) against the oracle: weighted draws are
integer decisions taken from the same float32 weights, so the drawn indices must equal
the oracle's exactly; the weight update is float32 arithmetic against the oracle's
float64 formula; the per-point losses of pifu_mlp_grad_ex against the oracle's BCE."""
import ctypes as C

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


@pytest.mark.parametrize("n,batch,seed,counter", [(1, 17, 3, 0), (4095, 300, 7, 2),
                                                  (4097, 1000, 11, 5), (300001, 4096, 5, 9)])
def test_draws_equal_the_oracle(pifu, n, batch, seed, counter):
    """Sizes around one scan tile (4096) and several tiles with a ragged tail."""
    from paper_2007_13988_amd.pifu import OhemSampler
    rng = np.random.default_rng(n)
    w = rng.uniform(1.0, 50.0, n).astype(np.float32)
    w[rng.integers(0, n, max(1, n // 100))] = 1e6     # a few hard points
    pool = torch.from_numpy(rng.uniform(-1, 1, (n, 4)).astype(np.float32)).cuda()
    s = OhemSampler(pool, batch, seed=seed)
    s.weights.copy_(torch.from_numpy(w))
    s.counter = counter
    pts = s.draw()
    torch.cuda.synchronize()
    print(f"[ohem] n={n} batch={batch}", flush=True)
    want = O.ohem_sample(w, batch, seed, counter)
    got = s.idx.cpu().numpy().astype(np.int64)
    assert np.array_equal(got, want)
    assert torch.equal(pts, pool[torch.from_numpy(want).cuda()])


def test_update_matches_eq6(pifu):
    from paper_2007_13988_amd.pifu import OhemSampler
    n, batch = 1000, 256
    pool = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    s = OhemSampler(pool, batch, alpha=0.7, beta=0.0)
    s.draw()
    torch.cuda.synchronize()
    idx = s.idx.cpu().numpy().astype(np.int64)
    # a point drawn twice has one loss (as in training, where its two copies are equal)
    L_point = np.linspace(0.0, 12.0, n).astype(np.float32)
    L = torch.from_numpy(L_point[idx]).cuda()
    s.update(L)
    torch.cuda.synchronize()
    want = O.ohem_point_weight(L_point[idx].astype(np.float64), 0.7, 0.0)
    got = s.weights.cpu().numpy().astype(np.float64)[idx]
    assert np.all(np.abs(got / want - 1.0) <= 2e-6), float(np.max(np.abs(got / want - 1.0)))
    untouched = np.setdiff1d(np.arange(n), idx)
    assert np.all(s.weights.cpu().numpy()[untouched] == 1.0)


def test_point_losses_match_the_oracle_bce(pifu):
    from paper_2007_13988_amd.train import MLPTrainer
    feat = synth.tiny_features()
    spec = synth.tiny_mlp()
    net = pifu.DeviceMLP(spec)
    rng = np.random.default_rng(4)
    n = 3000
    pts = np.concatenate([rng.uniform(-1, 1, (n, 3)), rng.uniform(0, 1, (n, 1))], 1).astype(np.float32)
    tr = MLPTrainer(net, n)
    pl = tr.point_loss(torch.from_numpy(feat).cuda(), torch.from_numpy(pts).cuda())
    torch.cuda.synchronize()
    s = O.field_logit(O.Field("mlp", feat=feat, mlp=spec), pts[:, :3].astype(np.float64))
    t = pts[:, 3].astype(np.float64)
    want = np.maximum(s, 0) - t * s + np.log1p(np.exp(-np.abs(s)))
    assert float(np.max(np.abs(pl.cpu().numpy() - want))) <= 1e-4
