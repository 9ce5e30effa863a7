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
    for t in (32, 64, 96, 256):
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


# ---------------------------------------------------------------- against the oracle

def test_batched_tiny_frames_match_oracle(pifu):
    """Every frame of a batched call against the FP64 oracle's localization: labels,
    cells and per-level statistics exact, occupancy within 1e-4."""
    import numpy as np
    from oracle import pifu_oracle as O
    from paper_2007_13988_amd.pifu import BatchedGrid
    spec = synth.tiny_mlp()
    net = pifu.DeviceMLP(spec)
    feats = [synth.feature_map(32, 32, 64, 4.0, 520 + f) for f in range(5)]
    finals = [5, 6, 5, 6, 4]
    fields = [pifu.DeviceField(pifu.FIELD_MLP, feat=F, mlp=net) for F in feats]
    bg = BatchedGrid(fields, [pifu.grid_opts(L, 3) for L in finals])
    bg.run()
    torch.cuda.synchronize()
    for i, (F, L) in enumerate(zip(feats, finals)):
        ref = O.occupancy_grid(O.Field("mlp", feat=F, mlp=spec), L, 3)
        b = bg.result(i)
        assert np.array_equal(b["labels"].cpu().numpy(), ref["labels"]), i
        assert b["n_cells"] == ref["cells"].size
        assert np.array_equal(b["cells"].cpu().numpy().astype(np.uint32), ref["cells"]), i
        assert np.max(np.abs(b["occ"].cpu().numpy() - ref["occ"])) <= 1e-4
        for g, rec in zip(b["stats"], ref["levels"]):
            for k in ("nodes", "b0", "dilated", "evaluated", "waves", "conflicts"):
                assert g[k] == rec.stats[k], (i, rec.level, k)


def test_batched_sixteen_ellipsoid_frames_256_and_512(pifu):
    """The batching workload's shape: 16 ellipsoid-union frames of uneven occupancy,
    final grids alternating 256^3 and 512^3, all from 32^3, in one call.  Every frame is
    bit-identical to its single call; four of them (two of each size) equal the FP64
    oracle exactly (analytic fields are evaluated in float64 on both sides)."""
    import numpy as np
    from oracle import pifu_oracle as O
    from paper_2007_13988_amd.pifu import BatchedGrid
    scales = [0.5 + 0.08 * i for i in range(16)]
    ells = [synth.ellipsoids(8, 500 + i, sc) for i, sc in enumerate(scales)]
    fields = [pifu.DeviceField.ellipsoids(e, 8.0) for e in ells]
    finals = [8 if i % 2 == 0 else 9 for i in range(16)]
    bg = BatchedGrid(fields, [pifu.grid_opts(L, 5) for L in finals])
    bg.run()
    torch.cuda.synchronize()
    print("[batched 16] ran", flush=True)
    occ = []
    for i in range(16):
        single = pifu.occupancy_grid(fields[i], finals[i], 5)
        b = bg.result(i)
        assert torch.equal(b["labels"], single["labels"]), i
        assert torch.equal(b["occ"], single["occ"]), i
        assert b["n_cells"] == single["n_cells"] and torch.equal(b["cells"], single["cells"]), i
        occ.append(float(b["labels"].float().mean().item()))
        del single
    print(f"[batched 16] occupied fraction {min(occ):.3f} .. {max(occ):.3f}", flush=True)
    assert min(occ) < 0.05 and max(occ) > 0.2
    for i in (0, 1, 14, 15):
        ref = O.occupancy_grid(O.Field("ellipsoids", ell=ells[i], sharpness=8.0), finals[i], 5)
        b = bg.result(i)
        assert np.array_equal(b["labels"].cpu().numpy(), ref["labels"]), i
        assert np.array_equal(b["cells"].cpu().numpy().astype(np.uint32), ref["cells"]), i
        for g, rec in zip(b["stats"], ref["levels"]):
            for k in ("nodes", "b0", "dilated", "evaluated", "waves", "conflicts"):
                assert g[k] == rec.stats[k], (i, rec.level, k)
        del ref


def test_batched_pifu_frames_256_match_oracle(pifu):
    """Eight PIFu-size MLP frames (different feature maps, one network) at 256^3 from
    32^3 in one call: bit-identical to single calls; frame 0 matches the oracle by the
    level-logic replay on the single call's evaluation map and by sampled nodes."""
    import numpy as np
    from oracle import pifu_oracle as O
    from paper_2007_13988_amd.pifu import BatchedGrid
    spec = synth.pifu_mlp()
    net = pifu.DeviceMLP(spec)
    feats = [synth.pifu_sequence(400 + f, 0) for f in range(8)]
    fields = [pifu.DeviceField(pifu.FIELD_MLP, feat=F, mlp=net) for F in feats]
    bg = BatchedGrid(fields, [pifu.grid_opts(8, 5) for _ in fields])
    bg.run()
    torch.cuda.synchronize()
    for i in range(8):
        single = pifu.occupancy_grid(fields[i], 8, 5, eval_level=(i == 0))
        b = bg.result(i)
        assert torch.equal(b["labels"], single["labels"]), i
        assert torch.equal(b["occ"], single["occ"]), i
        assert b["n_cells"] == single["n_cells"] and torch.equal(b["cells"], single["cells"]), i
        if i == 0:
            lab = single["labels"].cpu().numpy()
            evl = single["eval_level"].cpu().numpy()
            occ0 = single["occ"].cpu().numpy()
            cells0 = single["cells"].cpu().numpy().astype(np.uint32)
            stats0 = single["stats"]
        del single

    def lookup(P):
        idx = np.rint((P + 1.0) * 128.0).astype(np.int64)
        assert np.all(evl[idx[:, 0], idx[:, 1], idx[:, 2]] != 255)
        return np.where(lab[idx[:, 0], idx[:, 1], idx[:, 2]] == 1, 1.0, -1.0)

    res = O.localize(lookup, (8, 8, 8), 3)
    assert np.array_equal(res.label, lab)
    assert np.array_equal(O.eval_level_map(res), evl)
    assert np.array_equal(O.surface_cells(res.label), cells0)
    for rec, g in zip(res.levels, stats0):
        for k in ("nodes", "b0", "dilated", "evaluated", "waves", "conflicts"):
            assert g[k] == rec.stats[k], (rec.level, k)
    ev = np.argwhere(evl != 255)
    pick = ev[np.random.default_rng(7).choice(len(ev), 2000, replace=False)]
    ref = O.field_logit(O.Field("mlp", feat=feats[0], mlp=spec), -1.0 + 2.0 * pick / 256.0)
    assert np.array_equal(lab[pick[:, 0], pick[:, 1], pick[:, 2]], (ref > 0).astype(np.uint8))
    assert np.max(np.abs(occ0[pick[:, 0], pick[:, 1], pick[:, 2]] - O.sigmoid(ref))) <= 1e-4
