"""Precision ladder (BF16, FP16 and FP8 e4m3 MFMA with FP32 accumulation, FP32 re-run
of the points within 0.02 of p = 0.5, FP64 guard): operand conversions bit-checked
against torch's casts, probability error against the FP64 oracle on sampled points,
label flips, surface-cell agreement of the hierarchical grid, and the FP32 re-run of
FP16 evaluations whose values leave the binary16 range."""
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


def test_operand_conversions_match_torch_casts(pifu):
    from paper_2007_13988_amd.pifu import convert
    g = np.random.default_rng(0)
    x = np.concatenate([g.standard_normal(200000) * 50, g.uniform(-500, 500, 20000),
                        np.ldexp(1.0, np.arange(-14, 10)),
                        [0.0, 2.0 ** -10, 3 * 2.0 ** -10, 447.9, 448, 464, 1e6, -1e6]]).astype(np.float32)
    xt = torch.from_numpy(x)
    b = convert(xt, "bf16").cpu()
    assert torch.equal(b, xt.to(torch.bfloat16).view(torch.int16))
    h = convert(xt, "fp16").cpu()   # round to nearest even, overflow to infinity
    assert torch.equal(h, xt.to(torch.float16).view(torch.int16))
    f8 = convert(xt, "fp8").cpu()
    ref = xt.clamp(-448, 448).to(torch.float8_e4m3fn).view(torch.uint8)   # saturating reading
    assert torch.equal(f8, ref)


def _sample_points(fo, n_uniform, seed):
    """Half uniform, half jittered around nodes near the surface of the 33^3 grid."""
    g = O.occupancy_grid(fo, 5, 3)
    ev = np.argwhere(g["eval_level"] != 255)
    base = -1.0 + 2.0 * ev / 32
    near = synth.jitter_points(base[np.random.default_rng(seed).integers(0, len(base), n_uniform)],
                               2.0 / 32, seed + 1)
    pts = np.concatenate([synth.precision_points(n_uniform, seed), np.clip(near, -1, 1)])
    return pts.astype(np.float32).astype(np.float64)


def _dense_grid_points(L=5):
    n = (1 << L) + 1
    idx = np.arange(n ** 3)
    return O.lattice_coords((n, n, n), idx)


def _calibrated_tiny(pifu):
    """The tiny network with its static FP8 activation scales calibrated on the dense
    33^3 grid of the tiny workload (the library's FP32 pass)."""
    spec = synth.tiny_mlp()
    fg = pifu.DeviceField.mlp_field(synth.tiny_features(), spec)
    spec.fp8_amax = pifu.fp8_calibrate(fg, _dense_grid_points())
    return spec


def test_fp8_calibration_matches_oracle_layer_inputs(pifu):
    """The calibrated amax of every layer input equals max |input| of the FP64 forward
    pass over the same points (layer 0: the feature; later layers: the previous output
    and, with a skip, the feature)."""
    feat = synth.tiny_features()
    spec = synth.he_mlp(64, 1, [128, 64, 64, 1], [False, False, True, False], 221)
    fg = pifu.DeviceField.mlp_field(feat, spec)
    P = _dense_grid_points().astype(np.float32).astype(np.float64)
    got = pifu.fp8_calibrate(fg, P)
    f = O.bilinear_sample(feat, P[:, 0], P[:, 1])
    ins, pres = O.mlp_forward_cache(spec, f, P[:, 2:3])
    want = [np.max(np.abs(f))] + [np.max(np.abs(ins[l])) for l in range(1, len(spec.widths) - 1)]
    print("fp8 amax", got, want)
    assert np.allclose(got, want, rtol=1e-5, atol=0)


@pytest.mark.parametrize("prec,mean_tol", [("bf16", 5e-3), ("fp16", 1e-3), ("fp8", 3e-2)])
def test_probability_error_and_label_flips(pifu, prec, mean_tol):
    spec = _calibrated_tiny(pifu) if prec == "fp8" else synth.tiny_mlp()
    fo = O.Field("mlp", feat=synth.tiny_features(), mlp=synth.tiny_mlp())
    fg = pifu.DeviceField.mlp_field(synth.tiny_features(), spec)
    pts = _sample_points(fo, 500000, 403)
    ref = O.field_logit(fo, pts)
    p64 = O.sigmoid(ref)
    raw, _ = pifu.eval_points(fg, pts, precision=prec, band_delta=0.0, guard_logit=0.0)
    err = np.abs(O.sigmoid(raw.cpu().numpy().astype(np.float64)) - p64)
    lg, lab = pifu.eval_points(fg, pts, precision=prec, band_delta=0.02, guard_logit=1e-3)
    flips = int(np.sum(lab.cpu().numpy() != (ref > 0)))
    band = np.abs(p64 - 0.5) < 0.02
    print(f"{prec}: |p - p64| max {err.max():.3e} mean {err.mean():.3e} "
          f"p99 {np.quantile(err, 0.99):.3e}; label flips with band {flips} "
          f"of {pts.shape[0]}; points in band {int(band.sum())}")
    assert err.mean() < mean_tol
    # inside the band the label is decided in FP32/FP64, so any flip comes from a
    # low-precision error larger than the band itself: none for BF16; e4m3 keeps 3
    # mantissa bits and its logit error reaches past the band on ~0.1% of points
    assert flips <= (5e-3 if prec == "fp8" else 1e-4) * pts.shape[0]


# Surface-cell disagreement with the FP64 oracle on the tiny 33^3 grid.  With the band of
# the precision workload (|p - 0.5| < 0.02) BF16 and FP16 keep every label exact.  e4m3
# keeps 3 mantissa bits: with calibrated scales its logit error passes that band on a few
# dozen nodes, which moves 1.3% of the surface cells (measured), so its bound at 0.02 is
# 2%; a band sized to its error (0.1) brings it within the 0.1% bar.
CELL_CASES = [("bf16", 0.02, 1e-3), ("fp16", 0.02, 1e-3), ("fp8", 0.02, 2e-2),
              ("fp8", 0.1, 1e-3)]


@pytest.mark.parametrize("prec,band,bound", CELL_CASES)
def test_grid_surface_cells_against_oracle(pifu, prec, band, bound):
    from paper_2007_13988_amd.surrogate import cell_disagreement
    spec = _calibrated_tiny(pifu) if prec == "fp8" else synth.tiny_mlp()
    fo = O.Field("mlp", feat=synth.tiny_features(), mlp=synth.tiny_mlp())
    fg = pifu.DeviceField.mlp_field(synth.tiny_features(), spec)
    ref = O.occupancy_grid(fo, 5, 3)
    out = pifu.occupancy_grid(fg, 5, 3, precision=prec, band_delta=band)
    lab = out["labels"].cpu().numpy()
    d = cell_disagreement(out["cells"], torch.from_numpy(ref["cells"].astype(np.int64)).cuda())
    print(f"{prec} band {band}: label flips {int(np.sum(lab != ref['labels']))} of {lab.size}, "
          f"surface-cell disagreement {d:.2e}")
    assert d <= bound


def test_fp16_error_is_below_bf16(pifu):
    """binary16 keeps 3 more mantissa bits than bfloat16: its logit error is several
    times smaller on the same points, and a band of 0.005 leaves no label flip."""
    fo = O.Field("mlp", feat=synth.tiny_features(), mlp=synth.tiny_mlp())
    fg = pifu.DeviceField.mlp_field(synth.tiny_features(), synth.tiny_mlp())
    pts = _sample_points(fo, 200000, 405)
    ref = O.field_logit(fo, pts)
    err = {}
    for prec in ("bf16", "fp16"):
        raw, _ = pifu.eval_points(fg, pts, precision=prec, band_delta=0.0, guard_logit=0.0)
        err[prec] = np.abs(raw.cpu().numpy().astype(np.float64) - ref)
    print(f"logit error max bf16 {err['bf16'].max():.3e} fp16 {err['fp16'].max():.3e}; "
          f"mean bf16 {err['bf16'].mean():.3e} fp16 {err['fp16'].mean():.3e}")
    assert err["fp16"].mean() * 4 < err["bf16"].mean()
    assert err["fp16"].max() * 4 < err["bf16"].max()
    _, lab = pifu.eval_points(fg, pts, precision="fp16", band_delta=0.005, guard_logit=1e-3)
    assert int(np.sum(lab.cpu().numpy() != (ref > 0))) == 0


def _scaled(spec, s0, feat_scale=1.0):
    """The same function with layer 0's outputs scaled by s0 (undone by layer 1's weights
    of h0) and the features scaled by feat_scale (undone by every weight of f).  Powers
    of two: FP32 arithmetic on the scaled network is the original's, exactly."""
    import copy
    t = copy.deepcopy(spec)
    C = t.feat_dim
    t.W[0] = (t.W[0] * s0).astype(np.float32)
    t.W[0][:, :C] = (t.W[0][:, :C] / feat_scale).astype(np.float32)
    t.b[0] = (t.b[0] * s0).astype(np.float32)
    h0 = t.widths[0]
    t.W[1] = t.W[1].copy()
    t.W[1][:, :h0] = (t.W[1][:, :h0] / s0).astype(np.float32)
    for l in range(1, len(t.widths)):
        if t.skip[l]:
            t.W[l] = t.W[l].copy()
            t.W[l][:, -C:] = (t.W[l][:, -C:] / feat_scale).astype(np.float32)
    return t


@pytest.mark.parametrize("case", ["activation", "feature"])
def test_fp16_overflow_reruns_in_fp32(pifu, case):
    """Values outside the binary16 range (a hidden activation, or a sampled feature) send
    the call's evaluations to FP32: the results are those of the FP32 run, bit for bit."""
    spec = synth.he_mlp(64, 1, [128, 64, 1], [False, True, False], 207)
    feat = synth.tiny_features()
    if case == "activation":
        big, big_feat = _scaled(spec, 2.0 ** 17), feat
    else:
        big, big_feat = _scaled(spec, 1.0, 2.0 ** 17), (feat * 2.0 ** 17).astype(np.float32)
    f32 = pifu.DeviceField.mlp_field(feat, spec)
    f16 = pifu.DeviceField.mlp_field(big_feat, big)
    fo = O.Field("mlp", feat=feat, mlp=spec)
    pts = _sample_points(fo, 50000, 409)
    l32, b32 = pifu.eval_points(f32, pts, precision="fp32", guard_logit=1e-3)
    l16, b16 = pifu.eval_points(f16, pts, precision="fp16", band_delta=0.005, guard_logit=1e-3)
    assert torch.equal(b16, b32)
    assert torch.equal(l16, l32)
    g32 = pifu.occupancy_grid(f32, 6, 4, precision="fp32")
    g16 = pifu.occupancy_grid(f16, 6, 4, precision="fp16", band_delta=0.005)
    assert torch.equal(g16["labels"], g32["labels"])
    for s in g16["stats"]:
        assert s["band_fp32"] == s["mlp_points"]
    # the same networks unscaled stay in FP16 apart from the band
    g = pifu.occupancy_grid(f32, 6, 4, precision="fp16", band_delta=0.005)
    assert sum(s["band_fp32"] for s in g["stats"]) < 0.5 * sum(s["mlp_points"] for s in g["stats"])


@pytest.mark.parametrize("case", ["activation", "feature"])
def test_bf16_band_overflow_reruns_band_in_fp32(pifu, case):
    """A BF16 run re-evaluates its band on split-FP16 products.  A split operand outside the
    binary16 range (a hidden activation or a sampled feature, which BF16 itself holds) sends
    the band's points to FP32: points well inside the band then hold the FP32 run's logits
    bit for bit, where the unscaled network's band holds split-FP16 results.  Labels equal
    the FP32 run's, and the device-driven grid equals the blocking one."""
    spec = synth.he_mlp(64, 1, [128, 64, 1], [False, True, False], 207)
    feat = synth.tiny_features()
    if case == "activation":
        big, big_feat = _scaled(spec, 2.0 ** 17), feat
    else:
        big, big_feat = _scaled(spec, 1.0, 2.0 ** 17), (feat * 2.0 ** 17).astype(np.float32)
    f32 = pifu.DeviceField.mlp_field(feat, spec)
    fbig = pifu.DeviceField.mlp_field(big_feat, big)
    fo = O.Field("mlp", feat=feat, mlp=spec)
    pts = _sample_points(fo, 50000, 409)
    delta = 0.05
    kw = dict(precision="bf16", band_delta=delta, guard_logit=1e-3)
    l32, b32 = pifu.eval_points(f32, pts, precision="fp32", guard_logit=1e-3)
    lbig, bbig = pifu.eval_points(fbig, pts, **kw)
    lx3, bx3 = pifu.eval_points(f32, pts, **kw)
    assert torch.equal(bbig, b32) and torch.equal(bx3, b32)
    l32, lbig, lx3 = (t.cpu().numpy() for t in (l32, lbig, lx3))
    # BF16's logit error on this network stays far below a quarter of the band
    sure = (np.abs(l32) < 0.25 * np.log((0.5 + delta) / (0.5 - delta))) & (np.abs(l32) > 1e-3)
    print(f"{case}: {int(sure.sum())} points well inside the band", flush=True)
    assert sure.sum() > 100
    assert np.array_equal(lbig[sure], l32[sure])
    assert np.abs(lx3[sure] - l32[sure]).max() < 1e-4 and not np.array_equal(lx3[sure], l32[sure])
    g32 = pifu.occupancy_grid(f32, 6, 4, precision="fp32")
    gopt = dict(precision="bf16", band_delta=delta)
    gb = pifu.occupancy_grid(fbig, 6, 4, **gopt)
    assert torch.equal(gb["labels"], g32["labels"])
    ag = pifu.AsyncGrid(fbig, pifu.grid_opts(6, 4, **gopt))
    ag.run()
    torch.cuda.synchronize()
    r = ag.result()
    assert r["status"] == 0, r["status"]
    assert torch.equal(r["labels"], gb["labels"]) and torch.equal(r["occ"], gb["occ"])
    for sa, sb in zip(r["stats"], gb["stats"]):
        assert sa["band_fp32"] == sb["band_fp32"]


@pytest.mark.parametrize("net", ["tiny", "pifu"])
def test_fp16_band_products_are_fp32_accurate(pifu, net):
    """An FP16 run re-evaluates its band with FP32-accurate products of binary16 hi / lo
    operand splits (three FP16 MFMAs per step).  With the band covering every point the
    logits are those products: their error against the FP64 oracle stays within a small
    multiple of the FP32 path's and far below the FP64 guard (1e-3)."""
    if net == "tiny":
        feat, spec, n = synth.tiny_features(), synth.tiny_mlp(), 100000
    else:
        feat, spec, n = synth.pifu_sequence(102, 0), synth.pifu_mlp(), 6000
    fo = O.Field("mlp", feat=feat, mlp=spec)
    fg = pifu.DeviceField.mlp_field(feat, spec)
    pts = np.clip(synth.precision_points(n, 411) * 0.9, -1, 1).astype(np.float32).astype(np.float64)
    ref = O.field_logit(fo, pts)
    l32, _ = pifu.eval_points(fg, pts, precision="fp32", guard_logit=0.0, band_delta=0.0)
    lx3, _ = pifu.eval_points(fg, pts, precision="fp16", guard_logit=0.0, band_delta=0.5)
    e32 = np.abs(l32.cpu().numpy().astype(np.float64) - ref)
    ex3 = np.abs(lx3.cpu().numpy().astype(np.float64) - ref)
    print(f"{net}: logit error max FP32 {e32.max():.3e} split-FP16 {ex3.max():.3e}; "
          f"mean {e32.mean():.3e} / {ex3.mean():.3e}")
    assert ex3.max() < 1e-4
    assert ex3.max() < 8 * e32.max() + 1e-6
