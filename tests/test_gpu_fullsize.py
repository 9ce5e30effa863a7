"""Parity at the benchmarked size: 256^3 cells from 32^3 with the PIFu-size MLP, and the
512 x 512 x 256 render from 64 x 64 x 32 at yaw 90 -- the launch configuration that
bench.py times.

The FP64 oracle cannot evaluate all ~1.2 M points of a full frame in test time, so:
  * point values: sampled evaluated nodes are re-evaluated by the oracle (labels exact,
    occupancy within 1e-4);
  * level logic: the oracle's localization is replayed with the GPU's point labels as
    its "network"; it must request exactly the nodes the GPU evaluated at each level and
    reproduce the labels and surface cells bit for bit;
The render at the same size is replayed exactly in test_gpu_render_exact.py.
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


@pytest.fixture(scope="module")
def frame(pifu):
    feat = synth.pifu_features()
    spec = synth.pifu_mlp()
    fg = pifu.DeviceField.mlp_field(feat, spec)
    out = pifu.occupancy_grid(fg, 8, 5, eval_level=True)
    return dict(feat=feat, spec=spec, fg=fg, out={k: (v.cpu().numpy() if torch.is_tensor(v) else v)
                                                   for k, v in out.items()})


def test_sampled_evaluated_nodes_match_oracle(frame):
    out = frame["out"]
    ev = np.argwhere(out["eval_level"] != 255)
    rng = np.random.default_rng(5)
    pick = ev[rng.choice(len(ev), 3000, replace=False)]
    P = -1.0 + 2.0 * pick / 256.0
    fo = O.Field("mlp", feat=frame["feat"], mlp=frame["spec"])
    ref = O.field_logit(fo, P)
    got_lab = out["labels"][pick[:, 0], pick[:, 1], pick[:, 2]]
    got_occ = out["occ"][pick[:, 0], pick[:, 1], pick[:, 2]].astype(np.float64)
    assert np.array_equal(got_lab, (ref > 0).astype(np.uint8))
    assert np.max(np.abs(got_occ - O.sigmoid(ref))) <= 1e-4


def test_level_logic_replay_at_full_size(frame):
    out = frame["out"]
    lab = out["labels"]
    evl = out["eval_level"]

    def lookup(P):
        # every level's nodes are nodes of the 257^3 lattice
        idx = np.rint((P + 1.0) * 128.0).astype(np.int64)
        assert np.all(evl[idx[:, 0], idx[:, 1], idx[:, 2]] != 255), \
            "the oracle asked for a node the GPU never evaluated"
        return np.where(lab[idx[:, 0], idx[:, 1], idx[:, 2]] == 1, 1.0, -1.0)

    res = O.localize(lookup, (8, 8, 8), 3)
    assert np.array_equal(res.label, lab)
    assert np.array_equal(O.eval_level_map(res), evl)
    assert np.array_equal(O.surface_cells(res.label), out["cells"].astype(np.uint32))
    for rec, g in zip(res.levels, out["stats"]):
        for k in ("nodes", "b0", "dilated", "evaluated", "waves", "conflicts"):
            assert g[k] == rec.stats[k], (rec.level, k)
