"""The C ABI without a GPU: the library loads, exports every function include/pifu.h
declares, its structs match the ctypes mirrors, and host-side validation rejects bad
arguments before any launch."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pifu.h")


@pytest.fixture(scope="module")
def P():
    import paper_2007_13988_amd.pifu as P
    P.load_library()
    return P


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(pifu_\w+)\(", src, re.M)))


def test_library_exports_every_declared_function(P):
    lib = P.load_library()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True)
    for n in names:
        assert re.search(rf"\bT {n}\b", out.stdout), n


def test_struct_layouts_match_header(P):
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "pifu.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(pifu_mlp), sizeof(pifu_field), sizeof(pifu_level_stats),
         sizeof(pifu_grid_opts), sizeof(pifu_render_opts), sizeof(pifu_kernel_profile));
  printf("%zu %zu %zu\n", offsetof(pifu_field, feat), offsetof(pifu_field, ell),
         offsetof(pifu_mlp, fp8_amax));
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(pifu_grid_call), sizeof(pifu_render_call),
         offsetof(pifu_grid_call, n_cells), offsetof(pifu_grid_call, stream),
         offsetof(pifu_render_call, stats), offsetof(pifu_render_call, stream));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "s")
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(x) for x in lines[0].split()]
    assert sizes == [C.sizeof(P.PifuMLP), C.sizeof(P.PifuField), C.sizeof(P.PifuLevelStats),
                     C.sizeof(P.PifuGridOpts), C.sizeof(P.PifuRenderOpts),
                     C.sizeof(P.PifuKernelProfile)]
    offs = [int(x) for x in lines[1].split()]
    assert offs == [P.PifuField.feat.offset, P.PifuField.ell.offset, P.PifuMLP.fp8_amax.offset]
    calls = [int(x) for x in lines[2].split()]
    assert calls == [C.sizeof(P.PifuGridCall), C.sizeof(P.PifuRenderCall),
                     P.PifuGridCall.n_cells.offset, P.PifuGridCall.stream.offset,
                     P.PifuRenderCall.stats.offset, P.PifuRenderCall.stream.offset]


def _ell_field(P):
    return P.DeviceField.ellipsoids(synth.ellipsoids(8, 302), 8.0)


def _ws(P, field, opts):
    lib = P.load_library()
    n = C.c_size_t()
    st = lib.pifu_occupancy_grid_workspace_size(C.byref(field.struct) if field else None,
                                                C.byref(opts) if opts else None, C.byref(n))
    return st, n.value


def test_workspace_query_and_validation(P):
    f = _ell_field(P)
    st, n = _ws(P, f, P.grid_opts(8, 5))
    assert st == 0 and n > 257 ** 3
    assert _ws(P, f, P.grid_opts(10, 5))[0] == -1          # final grid too large
    assert _ws(P, f, P.grid_opts(5, 6))[0] == -1           # coarse finer than final
    assert _ws(P, f, P.grid_opts(5, 0))[0] == -1
    assert _ws(P, None, P.grid_opts(5, 3))[0] == -1        # null field
    assert _ws(P, f, None)[0] == -1                        # null options
    o = P.grid_opts(5, 3)
    o.precision = 7
    assert _ws(P, f, o)[0] == -1                           # unknown precision
    bad = P.DeviceField(P.FIELD_ELLIPSOIDS, ell=np.zeros((0, 12), np.float32))
    assert _ws(P, bad, P.grid_opts(5, 3))[0] == -1         # no ellipsoid


def test_render_workspace_validation(P):
    lib = P.load_library()
    f = _ell_field(P)
    n = C.c_size_t()
    o = P.render_opts(9, 8, 6)
    # the colour field must be an MLP field
    assert lib.pifu_render_view_workspace_size(C.byref(f.struct), C.byref(f.struct), C.byref(o),
                                               C.byref(n)) == -1
    o2 = P.render_opts(6, 2, 2)                            # z would have no coarse cells
    assert lib.pifu_render_view_workspace_size(C.byref(f.struct), C.byref(f.struct), C.byref(o2),
                                               C.byref(n)) == -1


def test_status_strings(P):
    lib = P.load_library()
    assert lib.pifu_status_string(0) == b"ok"
    assert lib.pifu_status_string(-2) == b"workspace too small"


def test_mlp_field_validation_checks_weight_pointers(P):
    """Host-side checks of a network descriptor (no device memory is touched: the
    workspace query validates before anything launches)."""
    from paper_2007_13988_amd.pifu import PifuField, PifuMLP
    widths = [128, 64, 1]
    m = PifuMLP()
    m.n_layers, m.feat_dim, m.n_extra = 3, 64, 1
    m.hidden_act, m.out_act = P.ACT["relu"], P.ACT["sigmoid"]
    for l, w in enumerate(widths):
        m.widths[l] = w
        m.W[l] = 0x100000 + 0x10000 * l      # stand-in addresses, 16-byte aligned
        m.b[l] = 0x200000 + 0x10000 * l
    f = PifuField()
    f.kind, f.H, f.W, f.C = P.FIELD_MLP, 32, 32, 64
    f.feat = 0x300000
    f.mlp = C.pointer(m)

    class _F:
        struct = f
    assert _ws(P, _F, P.grid_opts(5, 3))[0] == 0
    m.W[2] = 0x120004                          # misaligned head weights
    assert _ws(P, _F, P.grid_opts(5, 3))[0] == -1
    m.W[2] = 0x120000
    m.b[1] = 0                                 # null bias
    assert _ws(P, _F, P.grid_opts(5, 3))[0] == -1
    m.b[1] = 0x210000
    m.widths[0] = 96                           # hidden width not a multiple of 64
    assert _ws(P, _F, P.grid_opts(5, 3))[0] == -1


def test_grid_and_render_validates_both_calls_first(P):
    """pifu_grid_and_render checks both argument sets before either call starts; a
    rejected frame returns before the handle is touched, so a stand-in handle
    address serves here."""
    lib = P.load_library()
    f = _ell_field(P)
    go = P.grid_opts(5, 3)
    ro = P.render_opts(6, 5, 3)
    n_cells = C.c_uint32()
    v = (C.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    b = (C.c_float * 3)(0, 0, 0)
    _, gws = _ws(P, f, go)
    rws = C.c_size_t()
    assert lib.pifu_render_view_workspace_size(C.byref(f.struct), C.byref(f.struct), C.byref(ro),
                                               C.byref(rws)) == -1   # colour field must be an MLP
    col = P.PifuField()
    col.kind, col.H, col.W, col.C = P.FIELD_MLP, 32, 32, 64
    m = P.PifuMLP()
    m.n_layers, m.feat_dim, m.n_extra = 2, 64, 2
    m.hidden_act, m.out_act = P.ACT["relu"], P.ACT["tanh"]
    m.widths[0], m.widths[1] = 64, 3
    for l in range(2):
        m.W[l] = 0x100000 + 0x10000 * l
        m.b[l] = 0x200000 + 0x10000 * l
    col.feat = 0x300000
    col.mlp = C.pointer(m)
    assert lib.pifu_render_view_workspace_size(C.byref(f.struct), C.byref(col), C.byref(ro),
                                               C.byref(rws)) == 0
    fake = C.c_void_p(0x1000)   # stand-in device addresses (256-byte aligned); nothing launches

    def calls(gws_bytes=gws, rws_bytes=rws.value, occ=0x400000, rgb=0x500000):
        g = P.PifuGridCall(C.pointer(f.struct), C.pointer(go), occ, 0x410000, None, None, 0,
                           C.pointer(n_cells), None, 0x420000, gws_bytes, None)
        r = P.PifuRenderCall(C.pointer(f.struct), C.pointer(col), v, C.pointer(ro), b, rgb,
                             0x510000, 0x520000, None, 0x530000, rws_bytes, None)
        return g, r

    assert lib.pifu_grid_and_render(None, None, None) == -1
    g, r = calls()
    assert lib.pifu_grid_and_render(fake, None, C.byref(r)) == -1
    assert lib.pifu_grid_and_render(fake, C.byref(g), None) == -1
    g, r = calls(occ=0)                         # grid output missing
    assert lib.pifu_grid_and_render(fake, C.byref(g), C.byref(r)) == -1
    g, r = calls(rgb=0)                         # render output missing
    assert lib.pifu_grid_and_render(fake, C.byref(g), C.byref(r)) == -1
    g, r = calls(gws_bytes=gws - 1)
    assert lib.pifu_grid_and_render(fake, C.byref(g), C.byref(r)) == -2
    g, r = calls(rws_bytes=rws.value - 1)
    assert lib.pifu_grid_and_render(fake, C.byref(g), C.byref(r)) == -2


def test_cbn_field_validation_and_scope(P):
    """The CBN field's host-side checks (host stand-ins for the device arrays: the queries
    validate before anything touches memory): supported sizes pass, others are refused,
    and the calls outside its scope answer UNSUPPORTED."""
    lib = P.load_library()
    spec = synth.cbn_net(feat_dim=64, n_z=16, width=64, n_blocks=3, seed=1)
    feat = synth.feature_map(8, 8, 64, 2.0, 1)
    f = P.DeviceField.cbn_field(feat, spec, device="cpu")
    assert _ws(P, f, P.grid_opts(5, 3))[0] == 0
    for prec in ("bf16", "fp16", "fp8"):
        assert _ws(P, f, P.grid_opts(5, 3, precision=prec))[0] == -3, prec
    n = C.c_size_t()
    assert lib.pifu_occupancy_grid_async_workspace_size(C.byref(f.struct),
                                                        C.byref(P.grid_opts(5, 3)), 0,
                                                        C.byref(n)) == -3
    assert lib.pifu_eval_points_workspace_size(C.byref(f.struct), 0, 100, C.byref(n)) == 0
    assert lib.pifu_eval_points_workspace_size(C.byref(f.struct), 1, 100, C.byref(n)) == -3
    # sizes outside the supported set
    for field, bad in (("width", 96), ("n_z", 1), ("n_blocks", 9), ("n_blocks", 0),
                       ("feat_dim", 48)):
        old = getattr(f.cbn.struct, field)
        setattr(f.cbn.struct, field, bad)
        assert _ws(P, f, P.grid_opts(5, 3))[0] == -1, (field, bad)
        setattr(f.cbn.struct, field, old)
    f.cbn.struct.eps = 0.0
    assert _ws(P, f, P.grid_opts(5, 3))[0] == -1
    f.cbn.struct.eps = spec.eps
    f.cbn.struct.Wg[2] = None
    assert _ws(P, f, P.grid_opts(5, 3))[0] == -1
