"""Device-driven multi-frame batching (pifu_occupancy_grid_batched_async): every level
and conflict wave is one set of launches over all frames' combined work list, with every
count on the device, so the whole batch can be captured into one HIP graph.

Bar: every frame's labels, occupancy, cells and per-level statistics equal the blocking
batched call's and the frame's own pifu_occupancy_grid call's, bit for bit, eagerly and
on every replay of a captured graph; the status word is 0.
"""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

KEYS = ("nodes", "b0", "dilated", "evaluated", "waves", "conflicts", "mlp_points", "band_fp32",
        "guard_fp64")


@pytest.fixture(scope="module")
def pifu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_13988_amd as P
    P.load_library()
    return P


def _same(a, b, tag):
    assert torch.equal(a["labels"], b["labels"]), tag
    assert torch.equal(a["occ"], b["occ"]), tag
    assert a["n_cells"] == b["n_cells"], (tag, a["n_cells"], b["n_cells"])
    assert torch.equal(a["cells"], b["cells"]), tag
    for sa, sb in zip(a["stats"], b["stats"]):
        for k in KEYS:
            assert sa[k] == sb[k], (tag, sb["level"], k, sa[k], sb[k])


def _check(P, fields, finals, l0, max_points=0, **kw):
    singles = [P.occupancy_grid(f, L, l0, **kw) for f, L in zip(fields, finals)]
    most = max(s["waves"] for r in singles for s in r["stats"])
    print(f"[batched async] most conflict waves on a level: {most}", flush=True)
    # the default ladder has 12 waves; a longer loop runs with a cap it never reaches
    kw_a = dict(kw, max_waves=most) if most > 12 else kw
    opts = [P.grid_opts(L, l0, **kw_a) for L in finals]
    ab = P.AsyncBatchedGrid(fields, opts, max_points=max_points)
    ab.run()
    torch.cuda.synchronize()
    for i, single in enumerate(singles):
        r = ab.result(i)
        assert r["status"] == 0, r["status"]
        _same(r, single, f"frame {i}")
    return ab


def test_async_batched_tiny_mlp_frames(pifu):
    net = pifu.DeviceMLP(synth.tiny_mlp())
    fields = [pifu.DeviceField(pifu.FIELD_MLP, feat=synth.feature_map(32, 32, 64, 4.0, 500 + f),
                               mlp=net) for f in range(5)]
    print("[batched async] tiny MLP frames", flush=True)
    _check(pifu, fields, [5, 6, 5, 6, 4], 3)


def test_async_batched_ellipsoid_frames(pifu):
    fields = [pifu.DeviceField.ellipsoids(synth.ellipsoids(8, 600 + f), 8.0) for f in range(6)]
    print("[batched async] ellipsoid frames", flush=True)
    _check(pifu, fields, [6, 7, 6, 7, 6, 7], 4)


@pytest.mark.parametrize("prec,band", [("fp32", 0.0), ("fp16", 0.0075)])
def test_async_batched_pifu_frames(pifu, prec, band):
    """The benchmark's network on four frames of different feature maps, 256^3 from 32^3."""
    net = pifu.DeviceMLP(synth.pifu_mlp())
    fields = [pifu.DeviceField(pifu.FIELD_MLP, feat=synth.pifu_sequence(400 + f, 0), mlp=net)
              for f in range(4)]
    print(f"[batched async] PIFu frames {prec}", flush=True)
    _check(pifu, fields, [8, 8, 8, 8], 5, max_points=2 << 20, precision=prec, band_delta=band)


def test_async_batched_sixteen_frames_equal_blocking_batch(pifu):
    """The batching workload's shape: 16 ellipsoid-union frames of uneven occupancy, final
    grids alternating 256^3 and 512^3 from 32^3: equal to the blocking batched call."""
    from paper_2007_13988_amd.pifu import BatchedGrid
    scales = [0.5 + 0.08 * i for i in range(16)]
    fields = [pifu.DeviceField.ellipsoids(synth.ellipsoids(8, 500 + i, sc), 8.0)
              for i, sc in enumerate(scales)]
    finals = [8 if i % 2 == 0 else 9 for i in range(16)]
    opts = [pifu.grid_opts(L, 5) for L in finals]
    bg = BatchedGrid(fields, opts)
    bg.run()
    ab = pifu.AsyncBatchedGrid(fields, opts, max_points=24 << 20)
    ab.run()
    torch.cuda.synchronize()
    print("[batched async] 16 frames", flush=True)
    for i in range(16):
        r = ab.result(i)
        assert r["status"] == 0, r["status"]
        _same(r, bg.result(i), f"frame {i}")


def test_graph_capture_of_a_batch(pifu):
    """Four PIFu frames captured into one graph, replayed three times with eager work and
    synchronizations between replays: every replay equals the single calls."""
    net = pifu.DeviceMLP(synth.pifu_mlp())
    fields = [pifu.DeviceField(pifu.FIELD_MLP, feat=synth.pifu_sequence(410 + f, 0), mlp=net)
              for f in range(4)]
    finals = [8, 7, 8, 7]
    opts = [pifu.grid_opts(L, 5) for L in finals]
    refs = [pifu.occupancy_grid(f, L, 5) for f, L in zip(fields, finals)]
    ab = pifu.AsyncBatchedGrid(fields, opts, max_points=2 << 20)
    ab.run()   # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ab.run(torch.cuda.current_stream())
    for rep in range(3):
        for i in range(4):
            ab.occ[i].fill_(-1.0)
            ab.labels[i].zero_()
            ab.words[i].zero_()
        ab.status.fill_(77)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"[batched async] graph replay {rep}", flush=True)
        for i in range(4):
            r = ab.result(i)
            assert r["status"] == 0, (rep, r["status"])
            _same(r, refs[i], f"replay {rep} frame {i}")
        pifu.occupancy_grid(fields[0], 5, 3)   # eager work between replays
