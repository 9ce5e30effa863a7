"""GPU parity of the CBN + SoftZ lifting network (appendix, "Depth Representation" and
"Pixel-aligned 3D Lifting"; Tab. 2, HRNet-CBN-SoftZ) against the FP64 oracle, through the
C ABI: point evaluation, the hierarchical grid and the octree baseline with that network.

Bar: labels, evaluated sets, cells and per-level statistics bit-exact; FP32 occupancy
within 1e-4 of the FP64 value.  At the benchmarked size (256^3 from 32^3 on 256-channel
features) sampled evaluated nodes are re-evaluated by the oracle.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import pifu_oracle as O

pytestmark = pytest.mark.gpu

P_TOL = 1e-4


@pytest.fixture(scope="module")
def pifu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_13988_amd as P
    P.load_library()
    return P


def _tiny(P, n_blocks=3, seed=7):
    feat = synth.tiny_features()
    spec = synth.cbn_net(feat_dim=64, n_z=16, width=64, n_blocks=n_blocks, seed=seed,
                         out_bias=-1.0)
    return O.Field("cbn", feat=feat, mlp=spec), P.DeviceField.cbn_field(feat, spec)


def _paper(P, slab=False):
    """The paper-size network: random weights, or carrying the benchmark's depth slab."""
    feat = synth.pifu_features()
    spec = synth.pifu_cbn() if slab else synth.cbn_net()
    return O.Field("cbn", feat=feat, mlp=spec), P.DeviceField.cbn_field(feat, spec)


def _points(n, seed):
    pts = synth.precision_points(n, seed)
    pts[:50, :2] = np.clip(pts[:50, :2] * 1.3, -1.3, 1.3)   # some samples fall off the map
    pts[50:60, 2] = [-1.0, 1.0, -1.0, 1.0, 0.0, 1.0, -1.0, 0.5, -0.5, 1.0]   # depth-code ends
    pts[60:70, 2] = [-1.5, 1.5, -1.01, 1.01, -3.0, 3.0, -1.2, 1.2, -2.0, 2.0]   # clamped depths
    return pts.astype(np.float32).astype(np.float64)   # the ABI takes float32 points


def _eval_check(P, fo, fg, pts):
    lg, lab = P.eval_points(fg, pts)
    ref = O.field_logit(fo, pts)
    lg = lg.cpu().numpy().astype(np.float64)
    print(f"[cbn] max |logit diff| {np.max(np.abs(lg - ref)):.3g}", flush=True)
    assert np.max(np.abs(O.sigmoid(lg) - O.sigmoid(ref))) <= P_TOL
    assert np.array_equal(lab.cpu().numpy(), (ref > 0).astype(np.uint8))
    return lg, ref


def test_eval_points_tiny_cbn(pifu):
    fo, fg = _tiny(pifu)
    _eval_check(pifu, fo, fg, _points(20000, 31))


@pytest.mark.parametrize("n_blocks", [1, 2])
def test_eval_points_few_blocks(pifu, n_blocks):
    fo, fg = _tiny(pifu, n_blocks=n_blocks, seed=8 + n_blocks)
    _eval_check(pifu, fo, fg, _points(3000, 32 + n_blocks))


def test_eval_points_paper_size_cbn(pifu):
    fo, fg = _paper(pifu)
    lg, ref = _eval_check(pifu, fo, fg, _points(5000, 33))
    assert np.max(np.abs(lg - ref)) <= 1e-3


def test_guard_band_wider_than_every_logit(pifu):
    """Every point goes through the float64 re-evaluation: labels are the oracle's and the
    logits agree to float64 accumulation order."""
    fo, fg = _tiny(pifu)
    pts = _points(4000, 34)
    lg, lab = pifu.eval_points(fg, pts, guard_logit=1e9)
    ref = O.field_logit(fo, pts)
    assert np.array_equal(lab.cpu().numpy(), (ref > 0).astype(np.uint8))
    assert np.max(np.abs(lg.cpu().numpy().astype(np.float64) - ref)) <= 1e-5


def _grid_parity(gpu, ref):
    assert np.array_equal(gpu["labels"].cpu().numpy(), ref["labels"]), "labels differ"
    assert np.array_equal(gpu["eval_level"].cpu().numpy(), ref["eval_level"])
    assert gpu["n_cells"] == ref["cells"].size
    assert np.array_equal(gpu["cells"].cpu().numpy().astype(np.uint32), ref["cells"])
    occ = gpu["occ"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(occ - ref["occ"])) <= P_TOL
    for g, rec in zip(gpu["stats"], ref["levels"]):
        for k in ("nodes", "b0", "dilated", "evaluated", "waves", "conflicts"):
            assert g[k] == rec.stats[k], (rec.level, k, g[k], rec.stats[k])


@pytest.mark.parametrize("L,l0", [(5, 3), (6, 2)])
def test_grid_tiny_cbn(pifu, L, l0):
    fo, fg = _tiny(pifu)
    g = pifu.occupancy_grid(fg, L, l0, eval_level=True)
    ref = O.occupancy_grid(fo, L, l0)
    assert ref["cells"].size > 0 and ref["labels"].mean() > 0.02
    _grid_parity(g, ref)


@pytest.mark.parametrize("slab", [False, True])
def test_grid_paper_size_cbn_64(pifu, slab):
    fo, fg = _paper(pifu, slab)
    g = pifu.occupancy_grid(fg, 6, 4, eval_level=True)
    ref = O.occupancy_grid(fo, 6, 4)
    _grid_parity(g, ref)


def test_dense_grid_cbn(pifu):
    fo, fg = _tiny(pifu)
    g = pifu.occupancy_grid(fg, 4, 4, eval_level=True, dense=True)
    ref = O.occupancy_grid(fo, 4, 4)
    assert np.array_equal(g["labels"].cpu().numpy(), ref["labels"])
    assert np.max(np.abs(g["occ"].cpu().numpy().astype(np.float64) - ref["occ"])) <= P_TOL


def test_octree_binarized_cbn(pifu):
    fo, fg = _tiny(pifu)
    g = pifu.octree_grid(fg, 5, 3, "binarized", eval_level=True)
    o = O.octree_grid(fo, 5, 3, "binarized")
    assert np.array_equal(g["labels"].cpu().numpy(), o["labels"])
    assert np.array_equal(g["eval_level"].cpu().numpy(), o["eval_level"])
    assert g["n_cells"] == o["cells"].size


@pytest.mark.parametrize("slab", [False, True])
def test_sampled_nodes_at_benchmark_size(pifu, slab):
    """256^3 cells from 32^3 on the 256-channel features: sampled evaluated nodes."""
    fo, fg = _paper(pifu, slab)
    out = pifu.occupancy_grid(fg, 8, 5, eval_level=True)
    lab = out["labels"].cpu().numpy()
    occ = out["occ"].cpu().numpy()
    ev = np.argwhere(out["eval_level"].cpu().numpy() != 255)
    print(f"[cbn] 256^3: evaluated {len(ev)}, cells {out['n_cells']}", flush=True)
    assert out["n_cells"] > 0
    rng = np.random.default_rng(6)
    pick = ev[rng.choice(len(ev), 2000, replace=False)]
    P = -1.0 + 2.0 * pick / 256.0
    ref = O.field_logit(fo, P)
    assert np.array_equal(lab[pick[:, 0], pick[:, 1], pick[:, 2]], (ref > 0).astype(np.uint8))
    got = occ[pick[:, 0], pick[:, 1], pick[:, 2]].astype(np.float64)
    assert np.max(np.abs(got - O.sigmoid(ref))) <= P_TOL


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
def test_reduced_precision_is_unsupported(pifu, prec):
    _, fg = _tiny(pifu)
    with pytest.raises(RuntimeError, match="UNSUPPORTED|-3"):
        pifu.occupancy_grid(fg, 4, 3, precision=prec)
