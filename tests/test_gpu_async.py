"""Device-driven calls: pifu_occupancy_grid_async and pifu_render_view_async keep every
count on the device and read nothing back, so they can be captured into a HIP graph.

Bar: every output and every per-level statistic equals the blocking call's, bit for bit
(the same kernels in the same k order), eagerly and on every replay of a captured graph;
device-side conditions (a list longer than max_points, a capped wave ladder) arrive in
the status word.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

STAT_KEYS = ("nodes", "b0", "dilated", "evaluated", "waves", "conflicts", "mlp_points",
             "band_fp32", "guard_fp64", "surrogate_fallback", "shadow", "hits")


@pytest.fixture(scope="module")
def pifu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_13988_amd as P
    P.load_library()
    return P


def _same_grid(a, blocking):
    assert a["status"] == 0, a["status"]
    assert torch.equal(a["labels"], blocking["labels"])
    assert torch.equal(a["occ"], blocking["occ"])
    assert a["n_cells"] == blocking["n_cells"]
    assert torch.equal(a["cells"], blocking["cells"])
    for sa, sb in zip(a["stats"], blocking["stats"]):
        for k in STAT_KEYS:
            assert sa[k] == sb[k], (sb["level"], k, sa[k], sb[k])


def _fields(P, kind):
    if kind == "tiny":
        return P.DeviceField.mlp_field(synth.tiny_features(), synth.tiny_mlp()), (5, 3)
    if kind == "ell":
        return P.DeviceField.ellipsoids(synth.ellipsoids(8, 302), 8.0), (8, 5)
    return P.DeviceField.mlp_field(synth.pifu_sequence(102, 0), synth.pifu_mlp()), (8, 5)


@pytest.mark.parametrize("kind,prec,band", [("tiny", "fp32", 0.0), ("ell", "fp32", 0.0),
                                            ("pifu", "fp32", 0.0), ("pifu", "bf16", 0.02),
                                            ("pifu", "fp16", 0.0075)])
def test_async_grid_equals_blocking(pifu, kind, prec, band):
    fld, (L, l0) = _fields(pifu, kind)
    kw = dict(precision=prec, band_delta=band)
    blocking = pifu.occupancy_grid(fld, L, l0, **kw)
    ag = pifu.AsyncGrid(fld, pifu.grid_opts(L, l0, **kw))
    ag.run()
    torch.cuda.synchronize()
    print(f"[async grid] {kind} {prec}", flush=True)
    _same_grid(ag.result(), blocking)


def test_async_grid_with_surrogate_equals_blocking(pifu):
    """An untrained surrogate on the coarse levels: many fallbacks, same results."""
    feat = synth.pifu_sequence(102, 0)
    fld = pifu.DeviceField.mlp_field(feat, synth.pifu_mlp(), synth.surrogate_mlp())
    kw = dict(precision="fp16", band_delta=0.0075, surrogate_max_log2=6, surrogate_delta=0.3)
    blocking = pifu.occupancy_grid(fld, 8, 5, **kw)
    most = max(s["waves"] for s in blocking["stats"])
    print(f"[async surrogate] blocking call's most waves on a level: {most}", flush=True)
    # the default ladder (12 waves) either suffices or says it did not
    ag = pifu.AsyncGrid(fld, pifu.grid_opts(8, 5, **kw))
    ag.run()
    torch.cuda.synchronize()
    r = ag.result()
    assert bool(r["status"] & 2) == (most > 12), (r["status"], most)
    if most <= 12:
        _same_grid(r, blocking)
    # a ladder as long as the longest level's wave loop: the same results as the blocking
    # call (a cap that the blocking call never reaches changes nothing there)
    cap = max(most, 1)
    capped = pifu.occupancy_grid(fld, 8, 5, max_waves=cap, **kw)
    _same_grid_blocking(capped, blocking)
    ag = pifu.AsyncGrid(fld, pifu.grid_opts(8, 5, max_waves=cap, **kw))
    ag.run()
    torch.cuda.synchronize()
    r = ag.result()
    assert sum(s["surrogate_fallback"] for s in r["stats"]) > 0
    _same_grid(r, blocking)


def _same_grid_blocking(a, b):
    assert torch.equal(a["labels"], b["labels"]) and torch.equal(a["occ"], b["occ"])
    assert a["n_cells"] == b["n_cells"] and torch.equal(a["cells"], b["cells"])
    for sa, sb in zip(a["stats"], b["stats"]):
        for k in STAT_KEYS:
            assert sa[k] == sb[k], (sb["level"], k, sa[k], sb[k])


def pifu_color_field():
    import paper_2007_13988_amd as P
    return P.DeviceField.mlp_field(synth.color_features(), synth.color_mlp())


@pytest.mark.parametrize("prec,band", [("fp32", 0.0), ("fp16", 0.0075), ("bf16", 0.02)])
def test_async_render_equals_blocking(pifu, prec, band):
    fld, _ = _fields(pifu, "pifu")
    col = pifu_color_field()
    view = synth.yaw_view(90.0)
    kw = dict(precision=prec, band_delta=band)
    blocking = pifu.render_view(fld, col, view, 9, 8, 6, **kw)
    ar = pifu.AsyncRender(fld, col, view, (0.0, 0.0, 0.0), pifu.render_opts(9, 8, 6, **kw))
    ar.run()
    torch.cuda.synchronize()
    r = ar.result()
    print(f"[async render] {prec} status {r['status']}", flush=True)
    assert r["status"] == 0
    assert torch.equal(r["hit"], blocking["hit"])
    assert torch.equal(torch.nan_to_num(r["depth"], nan=-7.0),
                       torch.nan_to_num(blocking["depth"], nan=-7.0))
    assert torch.equal(r["rgb"], blocking["rgb"])
    for sa, sb in zip(r["stats"], blocking["stats"]):
        for k in STAT_KEYS:
            assert sa[k] == sb[k], (sb["level"], k, sa[k], sb[k])


def test_graph_capture_and_replay_of_a_frame(pifu):
    """Grid and render of one frame captured into one graph (the render on a second stream
    forked from the capture), replayed three times with eager work and synchronizations
    in between: every replay equals the blocking calls."""
    fld, _ = _fields(pifu, "pifu")
    col = pifu_color_field()
    view = synth.yaw_view(90.0)
    bg = (0.0, 0.0, 0.0)
    gb = pifu.occupancy_grid(fld, 8, 5)
    rb = pifu.render_view(fld, col, view, 9, 8, 6, bg)
    ag = pifu.AsyncGrid(fld, pifu.grid_opts(8, 5))
    ar = pifu.AsyncRender(fld, col, view, bg, pifu.render_opts(9, 8, 6))
    side = torch.cuda.Stream()
    # warm-up outside the capture (the handle and kernels are loaded)
    ag.run()
    ar.run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cur = torch.cuda.current_stream()
        side.wait_stream(cur)
        ag.run(cur)
        ar.run(side)
        cur.wait_stream(side)
    for rep in range(3):
        ag.occ.fill_(-1.0)
        ag.labels.zero_()
        ar.rgb.fill_(-5.0)
        ag.words.zero_()
        ar.words.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"[graph] replay {rep}", flush=True)
        _same_grid(ag.result(), gb)
        r = ar.result()
        assert r["status"] == 0
        assert torch.equal(r["hit"], rb["hit"]) and torch.equal(r["rgb"], rb["rgb"])
        for sa, sb in zip(r["stats"], rb["stats"]):
            for k in STAT_KEYS:
                assert sa[k] == sb[k], (rep, sb["level"], k)
        # eager work between replays
        pifu.occupancy_grid(fld, 5, 3)


def test_async_status_reports_list_over_and_capped_waves(pifu):
    fld, (L, l0) = _fields(pifu, "tiny")
    ag = pifu.AsyncGrid(fld, pifu.grid_opts(L, l0), max_points=1024)
    ag.run()
    torch.cuda.synchronize()
    assert ag.result()["status"] & 1          # a level's candidate list exceeds 1024 points
    capped = pifu.occupancy_grid(fld, L, l0, max_waves=1)
    ag = pifu.AsyncGrid(fld, pifu.grid_opts(L, l0, max_waves=1))
    ag.run()
    torch.cuda.synchronize()
    _same_grid(ag.result(), capped)
