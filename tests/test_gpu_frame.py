"""One frame through pifu_grid_and_render: the occupancy grid and the render of a
target view run concurrently (two host threads, two streams).  Every output and
statistic is bit-identical to pifu_occupancy_grid followed by pifu_render_view, and
on a tiny network the combined call meets the FP64 oracle as the single calls do."""
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


def _bits(t):
    """Bit pattern of a float tensor (NaN-safe exact comparison)."""
    return t.contiguous().view(torch.int32)


def _stats(st):
    return [s.as_dict() for s in st]


def _frame_outputs(P, fld, col, gkw, rkw, grid=(7, 4), render=(8, 7, 5)):
    gout = P.GridOutputs(fld, P.grid_opts(*grid, **gkw))
    rout = P.RenderOutputs(fld, col, P.render_opts(*render, **rkw))
    return gout, rout


def _assert_same(ga, ra, gb, rb):
    torch.cuda.synchronize()
    assert ga.n_cells.value == gb.n_cells.value
    n = min(ga.n_cells.value, ga.cells_cap)
    assert torch.equal(ga.cells[:n], gb.cells[:n])
    assert torch.equal(ga.labels, gb.labels)
    assert torch.equal(_bits(ga.occ), _bits(gb.occ))
    assert _stats(ga.stats) == _stats(gb.stats)
    assert torch.equal(ra.hit, rb.hit)
    assert torch.equal(_bits(ra.depth), _bits(rb.depth))
    assert torch.equal(_bits(ra.rgb), _bits(rb.rgb))
    assert _stats(ra.stats) == _stats(rb.stats)


FORMS = {
    "fp32": (dict(precision="fp32"), False),
    "fp16": (dict(precision="fp16", band_delta=0.0075), False),
    "surrogate_fp16": (dict(precision="fp16", band_delta=0.0075, surrogate_delta=0.3), True),
}


@pytest.mark.parametrize("form", list(FORMS))
def test_concurrent_frame_matches_separate_calls(pifu, form):
    kw, sur = FORMS[form]
    feat = synth.pifu_features(102)
    fld = pifu.DeviceField.mlp_field(feat, synth.pifu_mlp(),
                                     synth.surrogate_mlp() if sur else None)
    col = pifu.DeviceField.mlp_field(synth.color_features(), synth.color_mlp())
    view, bg = synth.yaw_view(90.0), (0.1, 0.2, 0.3)
    gkw, rkw = dict(kw), dict(kw)
    if sur:
        gkw["surrogate_max_log2"], rkw["surrogate_max_log2"] = 4, 5
    g1, r1 = _frame_outputs(pifu, fld, col, gkw, rkw)
    g2, r2 = _frame_outputs(pifu, fld, col, gkw, rkw)
    s1 = torch.cuda.current_stream()
    s2 = torch.cuda.Stream()
    pifu.occupancy_grid_into(fld, g1, s1)
    pifu.render_view_into(fld, col, view, bg, r1, s1)
    for rep in range(2):   # the second frame reuses outputs, workspaces and the second thread's state
        pifu.grid_and_render_into(fld, g2, col, view, bg, r2, s1, s2)
        _assert_same(g1, r1, g2, r2)
    assert int(r2.hit.sum()) > 0 and g2.n_cells.value > 0
    # the same stream for both: the calls run one after the other, same results
    g3, r3 = _frame_outputs(pifu, fld, col, gkw, rkw)
    pifu.grid_and_render_into(fld, g3, col, view, bg, r3, s1, s1)
    _assert_same(g1, r1, g3, r3)


def test_concurrent_frame_meets_oracle_tiny(pifu):
    feat, spec = synth.tiny_features(), synth.tiny_mlp()
    cfeat = synth.feature_map(32, 32, 64, 4.0, 5)
    cspec = synth.he_mlp(64, 2, [128, 64, 3], [False, False, False], 6, hidden_act="lrelu",
                         out_act="tanh")
    fo, co = O.Field("mlp", feat=feat, mlp=spec), O.Field("mlp", feat=cfeat, mlp=cspec)
    fg, cg = pifu.DeviceField.mlp_field(feat, spec), pifu.DeviceField.mlp_field(cfeat, cspec)
    view, bg = synth.yaw_view(45.0), (0.2, 0.4, 0.6)
    gout, rout = _frame_outputs(pifu, fg, cg, {}, {}, grid=(5, 3), render=(6, 5, 4))
    pifu.grid_and_render_into(fg, gout, cg, view, bg, rout, torch.cuda.current_stream(),
                              torch.cuda.Stream())
    torch.cuda.synchronize()
    gref = O.occupancy_grid(fo, 5, 3)
    assert np.array_equal(gout.labels.cpu().numpy(), gref["labels"])
    assert gout.n_cells.value == gref["cells"].size
    assert np.array_equal(gout.cells[:gout.n_cells.value].cpu().numpy().astype(np.uint32),
                          gref["cells"])
    occ = gout.occ.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(occ - gref["occ"])) <= 1e-4
    rref = O.render_view(fo, co, view, 6, 5, 4, bg)
    hit = rout.hit.cpu().numpy()
    assert np.array_equal(hit, rref["hit"])
    d = rout.depth.cpu().numpy()
    assert np.array_equal(np.isnan(d), np.isnan(rref["depth"]))
    assert np.max(np.abs(d[hit == 1] - rref["depth"][hit == 1])) <= 1e-4
    assert np.max(np.abs(rout.rgb.cpu().numpy() - rref["rgb"])) <= 1e-4


def test_profiler_counts_both_threads(pifu):
    """The render's launches (made by the second thread) are counted with the grid's."""
    fld = pifu.DeviceField.mlp_field(synth.pifu_features(102), synth.pifu_mlp())
    col = pifu.DeviceField.mlp_field(synth.color_features(), synth.color_mlp())
    view, bg = synth.yaw_view(90.0), (0.0, 0.0, 0.0)
    gout, rout = _frame_outputs(pifu, fld, col, {}, {})
    s1 = torch.cuda.current_stream()
    pifu.profile_enable(True)
    pifu.occupancy_grid_into(fld, gout, s1)
    pifu.render_view_into(fld, col, view, bg, rout, s1)
    sep = pifu.profile_read()
    pifu.profile_enable(True)
    pifu.grid_and_render_into(fld, gout, col, view, bg, rout, s1, torch.cuda.Stream())
    both = pifu.profile_read()
    pifu.profile_enable(False)
    assert sep["gemm_f32"]["launches"] > 0
    for k in sep:
        assert both[k]["launches"] == sep[k]["launches"], k
        assert both[k]["flops"] == pytest.approx(sep[k]["flops"]), k
        assert both[k]["total_ms"] > 0 or sep[k]["launches"] == 0, k


def test_concurrent_frame_dense_grid_with_eval_level(pifu):
    """The dense baseline grid with the per-node evaluation level, beside a render that
    returns no stats: both as the separate calls give them."""
    fld = pifu.DeviceField.mlp_field(synth.tiny_features(), synth.tiny_mlp())
    cfeat = synth.feature_map(32, 32, 64, 4.0, 5)
    cspec = synth.he_mlp(64, 2, [128, 64, 3], [False, False, False], 6, hidden_act="lrelu",
                         out_act="tanh")
    col = pifu.DeviceField.mlp_field(cfeat, cspec)
    view, bg = synth.yaw_view(30.0), (0.5, 0.5, 0.5)
    s1, s2 = torch.cuda.current_stream(), torch.cuda.Stream()

    def outs():
        g = pifu.GridOutputs(fld, pifu.grid_opts(6, 3, dense=True), eval_level=True)
        r = pifu.RenderOutputs(fld, col, pifu.render_opts(7, 6, 4))
        return g, r

    g1, r1 = outs()
    pifu.occupancy_grid_into(fld, g1, s1)
    pifu.render_view_into(fld, col, view, bg, r1, s1)
    g2, r2 = outs()
    lib = pifu.load_library()
    from paper_2007_13988_amd import pifu as PP
    import ctypes as C
    v = (C.c_float * 12)(*[float(x) for x in np.asarray(view, np.float32).reshape(-1)])
    b = (C.c_float * 3)(*bg)
    g = PP.PifuGridCall(C.pointer(fld.struct), C.pointer(g2.opts), g2.occ.data_ptr(),
                        g2.labels.data_ptr(), g2.eval_level.data_ptr(), g2.cells.data_ptr(),
                        g2.cells_cap, C.pointer(g2.n_cells),
                        C.cast(g2.stats, C.POINTER(PP.PifuLevelStats)), g2.ws.data_ptr(),
                        g2.ws_bytes, s1.cuda_stream)
    r = PP.PifuRenderCall(C.pointer(fld.struct), C.pointer(col.struct), v, C.pointer(r2.opts), b,
                          r2.rgb.data_ptr(), r2.depth.data_ptr(), r2.hit.data_ptr(), None,
                          r2.ws.data_ptr(), r2.ws_bytes, s2.cuda_stream)   # no render stats
    assert lib.pifu_grid_and_render(PP.context(), C.byref(g), C.byref(r)) == 0
    torch.cuda.synchronize()
    assert torch.equal(g1.eval_level, g2.eval_level)
    assert torch.equal(g1.labels, g2.labels)
    assert torch.equal(_bits(g1.occ), _bits(g2.occ))
    assert g1.n_cells.value == g2.n_cells.value
    assert _stats(g1.stats) == _stats(g2.stats)
    assert torch.equal(r1.hit, r2.hit) and int(r2.hit.sum()) > 0
    assert torch.equal(_bits(r1.depth), _bits(r2.depth))
    assert torch.equal(_bits(r1.rgb), _bits(r2.rgb))


def test_concurrent_frame_full_size_matches_separate_calls(pifu):
    """The benchmark's sizes and launch configuration: a 256^3 grid from 32^3 and a
    512 x 512 x 256 render from 64 x 64 x 32 on the PIFu-size network, FP16 with the
    split-FP16 band.  The concurrent frame equals the two calls bit for bit."""
    fld = pifu.DeviceField.mlp_field(synth.pifu_sequence(102, 0), synth.pifu_mlp())
    col = pifu.DeviceField.mlp_field(synth.color_features(), synth.color_mlp())
    view, bg = synth.yaw_view(90.0), (0.0, 0.0, 0.0)
    kw = dict(precision="fp16", band_delta=0.0075, guard_logit=1e-3)
    g1, r1 = _frame_outputs(pifu, fld, col, kw, kw, grid=(8, 5), render=(9, 8, 6))
    g2, r2 = _frame_outputs(pifu, fld, col, kw, kw, grid=(8, 5), render=(9, 8, 6))
    s1, s2 = torch.cuda.current_stream(), torch.cuda.Stream()
    pifu.occupancy_grid_into(fld, g1, s1)
    pifu.render_view_into(fld, col, view, bg, r1, s1)
    pifu.grid_and_render_into(fld, g2, col, view, bg, r2, s1, s2)
    _assert_same(g1, r1, g2, r2)
    assert g2.n_cells.value > 100000 and int(r2.hit.sum()) > 50000
