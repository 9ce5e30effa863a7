"""Multi-frame batching: results of pifu_occupancy_grid_batched are bit-identical to
one pifu_occupancy_grid call per frame (labels, occupancy, cells, per-level stats)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pifu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_13988_amd as P
    P.load_library()
    return P


def _same(P, fields, finals, l0, **kw):
    from paper_2007_13988_amd.pifu import BatchedGrid
    opts = [P.grid_opts(L, l0, **kw) for L in finals]
    bg = BatchedGrid(fields, opts)
    bg.run()
    torch.cuda.synchronize()
    for i, (f, L) in enumerate(zip(fields, finals)):
        single = P.occupancy_grid(f, L, l0, **kw)
        b = bg.result(i)
        assert torch.equal(b["labels"], single["labels"]), i
        assert torch.equal(b["occ"], single["occ"]), i
        assert b["n_cells"] == single["n_cells"]
        assert torch.equal(b["cells"], single["cells"]), i
        for sb, ss in zip(b["stats"], single["stats"]):
            for k in ("nodes", "b0", "dilated", "evaluated", "waves", "conflicts", "mlp_points",
                      "guard_fp64"):
                assert sb[k] == ss[k], (i, k, sb[k], ss[k])


def test_batched_mlp_frames_match_single_calls(pifu):
    spec = synth.tiny_mlp()
    net = pifu.DeviceMLP(spec)
    fields = [pifu.DeviceField(pifu.FIELD_MLP, feat=synth.feature_map(32, 32, 64, 4.0, 500 + f),
                               mlp=net) for f in range(5)]
    _same(pifu, fields, [5, 6, 5, 6, 4], 3)


def test_batched_ellipsoid_frames_match_single_calls(pifu):
    fields = [pifu.DeviceField.ellipsoids(synth.ellipsoids(8, 600 + f), 8.0) for f in range(6)]
    _same(pifu, fields, [6, 7, 6, 7, 6, 7], 4)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_tile_choice_never_changes_results(pifu, prec):
    """Forced point tiles 32/64/128/256 and the autotuned choice give identical grids."""
    from paper_2007_13988_amd import pifu as PP
    feat = synth.pifu_features(513)
    spec = synth.pifu_mlp()
    fld = pifu.DeviceField.mlp_field(feat, spec)
    ref = pifu.occupancy_grid(fld, 6, 4, precision=prec, tile_m=128)
    for t in (32, 64, 256):
        o = pifu.occupancy_grid(fld, 6, 4, precision=prec, tile_m=t)
        assert torch.equal(o["labels"], ref["labels"]) and torch.equal(o["occ"], ref["occ"]), t
    chosen = PP.autotune(fld, prec, batch_sizes=(4096, 16384))
    assert all(c in (64, 128, 256) for v in chosen.values() for c in v) and chosen[4096]
    o = pifu.occupancy_grid(fld, 6, 4, precision=prec)
    assert torch.equal(o["labels"], ref["labels"]) and torch.equal(o["occ"], ref["occ"])
    PP.autotune_clear()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_batched_pifu_frames_match_single_calls(pifu, prec):
    spec = synth.pifu_mlp()
    net = pifu.DeviceMLP(spec)
    fields = [pifu.DeviceField(pifu.FIELD_MLP, feat=synth.feature_map(128, 128, 256, 16.0, 510 + f),
                               mlp=net) for f in range(3)]
    _same(pifu, fields, [6, 7, 6], 4, precision=prec)
