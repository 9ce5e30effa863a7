"""ctypes binding of libpifu (include/pifu.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels of
libpifu.so.  PyTorch provides device memory (outputs, workspace, weights) and the
current stream.  There is no CPU fallback: without the built library every call
raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpifu.so")
INCLUDE = os.path.join(os.path.dirname(_HERE), "include", "pifu.h")

MAX_LAYERS = 8
CBN_MAX_BLOCKS = 8
FIELD_MLP, FIELD_ELLIPSOIDS, FIELD_PLANE, FIELD_CBN = 0, 1, 2, 3
ACT = {"relu": 1, "lrelu": 2, "sigmoid": 3, "tanh": 4}
PREC = {"fp32": 0, "bf16": 1, "fp8": 2, "fp16": 3}
STATUS = {0: "ok", -1: "invalid argument", -2: "workspace too small", -3: "unsupported",
          -4: "HIP runtime error", -5: "scratch too small (no-allocation entry point)"}


class PifuMLP(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("feat_dim", C.c_int32), ("n_extra", C.c_int32),
                ("hidden_act", C.c_int32), ("out_act", C.c_int32),
                ("widths", C.c_int32 * MAX_LAYERS), ("skip", C.c_int32 * MAX_LAYERS),
                ("W", C.c_void_p * MAX_LAYERS), ("b", C.c_void_p * MAX_LAYERS),
                ("fp8_amax", C.c_float * MAX_LAYERS)]


class PifuCBN(C.Structure):
    _fields_ = [("feat_dim", C.c_int32), ("n_z", C.c_int32), ("width", C.c_int32),
                ("n_blocks", C.c_int32), ("eps", C.c_float), ("Wp", C.c_void_p), ("bp", C.c_void_p)] + \
               [(k, C.c_void_p * CBN_MAX_BLOCKS) for k in ("W", "b", "Wg", "bg", "Wb", "bb", "mean",
                                                          "var")] + \
               [("Wo", C.c_void_p), ("bo", C.c_void_p)]


class PifuField(C.Structure):
    _fields_ = [("kind", C.c_int32), ("H", C.c_int32), ("W", C.c_int32), ("C", C.c_int32),
                ("feat", C.c_void_p), ("mlp", C.POINTER(PifuMLP)),
                ("surrogate", C.POINTER(PifuMLP)), ("n_ell", C.c_int32),
                ("sharpness", C.c_float), ("ell", C.c_void_p), ("plane", C.c_float * 4),
                ("cbn", C.POINTER(PifuCBN))]


class PifuLevelStats(C.Structure):
    _fields_ = [("level", C.c_int32), ("nodes", C.c_uint32), ("b0", C.c_uint32),
                ("dilated", C.c_uint32), ("evaluated", C.c_uint32), ("waves", C.c_uint32),
                ("conflicts", C.c_uint32), ("mlp_points", C.c_uint32), ("band_fp32", C.c_uint32),
                ("guard_fp64", C.c_uint32), ("surrogate_fallback", C.c_uint32),
                ("shadow", C.c_uint32), ("hits", C.c_uint32), ("reserved", C.c_uint32 * 3)]

    def as_dict(self) -> Dict[str, int]:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class PifuGridOpts(C.Structure):
    _fields_ = [("log2_final", C.c_int32), ("log2_coarse", C.c_int32), ("dense", C.c_int32),
                ("precision", C.c_int32), ("band_delta", C.c_float), ("guard_logit", C.c_float),
                ("surrogate_max_log2", C.c_int32), ("surrogate_delta", C.c_float),
                ("tile_m", C.c_int32), ("max_waves", C.c_int32)]


class PifuRenderOpts(C.Structure):
    _fields_ = [("log2_w", C.c_int32), ("log2_d", C.c_int32), ("log2_coarse_w", C.c_int32),
                ("precision", C.c_int32), ("band_delta", C.c_float), ("guard_logit", C.c_float),
                ("surrogate_max_log2", C.c_int32), ("surrogate_delta", C.c_float),
                ("tile_m", C.c_int32), ("max_waves", C.c_int32)]


class PifuGridOut(C.Structure):
    _fields_ = [("occ", C.c_void_p), ("labels", C.c_void_p), ("cells", C.c_void_p),
                ("cells_cap", C.c_uint32), ("n_cells", C.c_uint32),
                ("stats", C.POINTER(PifuLevelStats))]


class PifuGridOutDev(C.Structure):
    _fields_ = [("occ", C.c_void_p), ("labels", C.c_void_p), ("cells", C.c_void_p),
                ("cells_cap", C.c_uint32), ("n_cells_dev", C.c_void_p), ("stats_dev", C.c_void_p)]


class PifuGridCall(C.Structure):
    _fields_ = [("field", C.POINTER(PifuField)), ("opts", C.POINTER(PifuGridOpts)),
                ("occ", C.c_void_p), ("labels", C.c_void_p), ("eval_level", C.c_void_p),
                ("cells", C.c_void_p), ("cells_cap", C.c_uint32),
                ("n_cells", C.POINTER(C.c_uint32)), ("stats", C.POINTER(PifuLevelStats)),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stream", C.c_void_p)]


class PifuRenderCall(C.Structure):
    _fields_ = [("occ_field", C.POINTER(PifuField)), ("color_field", C.POINTER(PifuField)),
                ("view", C.POINTER(C.c_float)), ("opts", C.POINTER(PifuRenderOpts)),
                ("bg", C.POINTER(C.c_float)), ("rgb", C.c_void_p), ("depth", C.c_void_p),
                ("hit", C.c_void_p), ("stats", C.POINTER(PifuLevelStats)),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stream", C.c_void_p)]


class PifuRenderTrace(C.Structure):
    _fields_ = [("kstar", C.c_void_p), ("k1", C.c_void_p), ("eval_level", C.c_void_p),
                ("logit", C.c_void_p)]


class PifuKernelProfile(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("total_ms", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


KERN = {"gemm_f32": 0, "gemm_bf16": 1, "gemm_fp8": 2, "gather": 3, "head": 4, "gemm_f16": 5,
        "gemm_f16x3": 6}
KERN_COUNT = 8

EXPORTS = ["pifu_create", "pifu_destroy", "pifu_status_string",
           "pifu_occupancy_grid_workspace_size", "pifu_occupancy_grid",
           "pifu_render_view_workspace_size", "pifu_render_view",
           "pifu_eval_points_workspace_size", "pifu_eval_points",
           "pifu_profile_enable", "pifu_profile_read", "pifu_mlp_train_workspace_size",
           "pifu_mlp_grad", "pifu_rmsprop_step", "pifu_occupancy_grid_batched_workspace_size",
           "pifu_occupancy_grid_batched", "pifu_autotune_mlp", "pifu_autotune_clear",
           "pifu_convert_f32", "pifu_grid_and_render", "pifu_render_view_traced", "pifu_fp8_calibrate",
           "pifu_occupancy_grid_async_workspace_size", "pifu_occupancy_grid_async",
           "pifu_render_view_async_workspace_size", "pifu_render_view_async",
           "pifu_noalloc_scratch_bytes", "pifu_occupancy_grid_async_noalloc", "pifu_octree_grid",
           "pifu_occupancy_grid_batched_async_workspace_size", "pifu_occupancy_grid_batched_async",
           "pifu_mlp_grad_ex", "pifu_ohem_sample_workspace_size", "pifu_ohem_sample",
           "pifu_ohem_update", "pifu_mesh_workspace_size", "pifu_mesh"]

_lib = None


def load_library():
    """Loads libpifu.so and declares the C signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32, u32, sz = C.c_int32, C.c_uint32, C.c_size_t
    lib.pifu_create.argtypes = [C.POINTER(P)]
    lib.pifu_destroy.argtypes = [P]
    lib.pifu_destroy.restype = None
    lib.pifu_status_string.argtypes = [i32]
    lib.pifu_status_string.restype = C.c_char_p
    lib.pifu_occupancy_grid_workspace_size.argtypes = [C.POINTER(PifuField),
                                                       C.POINTER(PifuGridOpts), C.POINTER(sz)]
    lib.pifu_occupancy_grid.argtypes = [P, C.POINTER(PifuField), C.POINTER(PifuGridOpts), P, P, P,
                                        P, u32, C.POINTER(u32), C.POINTER(PifuLevelStats), P, sz, P]
    lib.pifu_render_view_workspace_size.argtypes = [C.POINTER(PifuField), C.POINTER(PifuField),
                                                    C.POINTER(PifuRenderOpts), C.POINTER(sz)]
    lib.pifu_render_view.argtypes = [P, C.POINTER(PifuField), C.POINTER(PifuField),
                                     C.POINTER(C.c_float), C.POINTER(PifuRenderOpts),
                                     C.POINTER(C.c_float), P, P, P, C.POINTER(PifuLevelStats), P,
                                     sz, P]
    lib.pifu_render_view_traced.argtypes = [P, C.POINTER(PifuField), C.POINTER(PifuField),
                                            C.POINTER(C.c_float), C.POINTER(PifuRenderOpts),
                                            C.POINTER(C.c_float), P, P, P,
                                            C.POINTER(PifuLevelStats), P, sz, P,
                                            C.POINTER(PifuRenderTrace)]
    lib.pifu_fp8_calibrate.argtypes = [P, C.POINTER(PifuField), P, u32, C.POINTER(C.c_float), P,
                                       sz, P]
    lib.pifu_occupancy_grid_async_workspace_size.argtypes = [C.POINTER(PifuField),
                                                             C.POINTER(PifuGridOpts), u32,
                                                             C.POINTER(sz)]
    lib.pifu_occupancy_grid_async.argtypes = [P, C.POINTER(PifuField), C.POINTER(PifuGridOpts), u32,
                                              P, P, P, P, u32, P, P, P, P, sz, P]
    lib.pifu_octree_grid.argtypes = [P, C.POINTER(PifuField), C.POINTER(PifuGridOpts), i32,
                                     C.c_double, P, P, P, P, u32, C.POINTER(u32),
                                     C.POINTER(PifuLevelStats), P, sz, P]
    lib.pifu_occupancy_grid_batched_async_workspace_size.argtypes = [i32, C.POINTER(C.c_void_p),
                                                                     C.POINTER(C.c_void_p), u32,
                                                                     C.POINTER(sz)]
    lib.pifu_occupancy_grid_batched_async.argtypes = [P, i32, C.POINTER(C.c_void_p),
                                                      C.POINTER(C.c_void_p), u32,
                                                      C.POINTER(PifuGridOutDev), P, P, sz, P]
    lib.pifu_mlp_grad_ex.argtypes = [P, C.POINTER(PifuField), P, u32, C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), P, P, P, sz, P]
    lib.pifu_ohem_sample_workspace_size.argtypes = [u32, C.POINTER(sz)]
    lib.pifu_ohem_sample.argtypes = [P, P, u32, P, u32, C.c_uint64, C.c_uint64, P, P, P, sz, P]
    lib.pifu_ohem_update.argtypes = [P, P, P, u32, C.c_float, C.c_float, P, P]
    lib.pifu_mesh_workspace_size.argtypes = [i32, u32, u32, C.POINTER(PifuField), C.POINTER(sz)]
    lib.pifu_mesh.argtypes = [P, i32, P, P, P, u32, C.POINTER(PifuField), P, i32, i32, P, P, u32,
                              C.POINTER(u32), P, u32, C.POINTER(u32), P, sz, P]
    lib.pifu_noalloc_scratch_bytes.argtypes = []
    lib.pifu_occupancy_grid_async_noalloc.argtypes = [P, C.POINTER(PifuField),
                                                      C.POINTER(PifuGridOpts), u32, P, P, P, P,
                                                      u32, P, P, P, P]
    lib.pifu_render_view_async_workspace_size.argtypes = [C.POINTER(PifuField),
                                                          C.POINTER(PifuField),
                                                          C.POINTER(PifuRenderOpts), u32,
                                                          C.POINTER(sz)]
    lib.pifu_render_view_async.argtypes = [P, C.POINTER(PifuField), C.POINTER(PifuField),
                                           C.POINTER(C.c_float), C.POINTER(PifuRenderOpts), u32,
                                           C.POINTER(C.c_float), P, P, P, P, P, P, sz, P]
    lib.pifu_eval_points_workspace_size.argtypes = [C.POINTER(PifuField), i32, u32, C.POINTER(sz)]
    lib.pifu_eval_points.argtypes = [P, C.POINTER(PifuField), i32, C.c_float, C.c_float, P, u32, P,
                                     P, P, P, sz, P]
    PP = C.POINTER(C.c_void_p)
    lib.pifu_mlp_train_workspace_size.argtypes = [C.POINTER(PifuField), u32, C.POINTER(sz)]
    lib.pifu_mlp_grad.argtypes = [P, C.POINTER(PifuField), P, u32, PP, PP, P, P, sz, P]
    lib.pifu_rmsprop_step.argtypes = [P, C.POINTER(PifuMLP), PP, PP, PP, PP, C.c_float, C.c_float,
                                      C.c_float, P]
    lib.pifu_occupancy_grid_batched_workspace_size.argtypes = [i32, PP, PP, C.POINTER(sz)]
    lib.pifu_occupancy_grid_batched.argtypes = [P, i32, PP, PP, C.POINTER(PifuGridOut), P, sz, P]
    lib.pifu_autotune_mlp.argtypes = [P, C.POINTER(PifuField), i32, u32, C.POINTER(i32), P, sz, P]
    lib.pifu_autotune_clear.argtypes = [P]
    lib.pifu_convert_f32.argtypes = [P, P, u32, i32, P, P]
    lib.pifu_grid_and_render.argtypes = [P, C.POINTER(PifuGridCall), C.POINTER(PifuRenderCall)]
    lib.pifu_profile_enable.argtypes = [P, i32]
    lib.pifu_profile_read.argtypes = [P, C.POINTER(PifuKernelProfile)]
    for name in EXPORTS:
        if name not in ("pifu_destroy", "pifu_status_string", "pifu_noalloc_scratch_bytes"):
            getattr(lib, name).restype = i32
    lib.pifu_noalloc_scratch_bytes.restype = sz
    _lib = lib
    return lib


class PifuError(RuntimeError):
    pass


def _check(status: int, what: str):
    if status != 0:
        raise PifuError(f"{what} failed: {STATUS.get(status, status)} ({status})")


_ctx: Dict[int, C.c_void_p] = {}


def context() -> C.c_void_p:
    dev = torch.cuda.current_device()
    if dev not in _ctx:
        lib = load_library()
        h = C.c_void_p()
        _check(lib.pifu_create(C.byref(h)), "pifu_create")
        _ctx[dev] = h
    return _ctx[dev]


def autotune(field: "DeviceField", precision="fp32", batch_sizes=(4096, 16384, 65536),
             stream=None) -> Dict[int, List[int]]:
    """Runs the library's tile autotuner for each batch-size bucket; returns the
    chosen point tile per timed layer for each batch size."""
    lib = load_library()
    out = {}
    for m in batch_sizes:
        sz = C.c_size_t()
        _check(lib.pifu_eval_points_workspace_size(C.byref(field.struct), PREC[precision], m,
                                                   C.byref(sz)), "autotune workspace")
        ws = torch.empty(sz.value, dtype=torch.uint8, device="cuda")
        chosen = (C.c_int32 * 16)(*([0] * 16))
        _check(lib.pifu_autotune_mlp(context(), C.byref(field.struct), PREC[precision], m, chosen,
                                     ws.data_ptr(), sz.value, _stream(stream)), "pifu_autotune_mlp")
        out[m] = [c for c in chosen if c]
    return out


def convert(x: torch.Tensor, precision: str) -> torch.Tensor:
    """The library's bf16 / fp16 / e4m3 conversion of a device float32 tensor (raw bits)."""
    x = x.contiguous().to(device="cuda", dtype=torch.float32)
    out = torch.empty(x.numel(), dtype=torch.int16 if precision in ("bf16", "fp16") else torch.uint8,
                      device="cuda")
    _check(load_library().pifu_convert_f32(context(), x.data_ptr(), x.numel(), PREC[precision],
                                           out.data_ptr(), _stream(None)), "pifu_convert_f32")
    return out


def autotune_clear() -> None:
    _check(load_library().pifu_autotune_clear(context()), "pifu_autotune_clear")


def profile_enable(on: bool = True) -> None:
    """Turns the library's per-launch event timing on/off (resets the accumulators)."""
    _check(load_library().pifu_profile_enable(context(), int(on)), "pifu_profile_enable")


def profile_read() -> Dict[str, Dict[str, float]]:
    recs = (PifuKernelProfile * KERN_COUNT)()
    _check(load_library().pifu_profile_read(context(), recs), "pifu_profile_read")
    return {name: dict(launches=recs[i].launches, total_ms=recs[i].total_ms,
                       flops=recs[i].flops, bytes=recs[i].bytes) for name, i in KERN.items()}


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ device-side inputs

class DeviceMLP:
    """An MLP whose weights live on the GPU, described for the C ABI."""

    def __init__(self, spec, device="cuda"):
        self.spec = spec
        self.W = [torch.as_tensor(np.ascontiguousarray(w, np.float32)).to(device) for w in spec.W]
        self.b = [torch.as_tensor(np.ascontiguousarray(b, np.float32)).to(device) for b in spec.b]
        s = PifuMLP()
        s.n_layers = len(spec.widths)
        s.feat_dim = spec.feat_dim
        s.n_extra = spec.n_extra
        s.hidden_act = ACT[spec.hidden_act]
        s.out_act = ACT[spec.out_act]
        for l, w in enumerate(spec.widths):
            s.widths[l] = w
            s.skip[l] = int(bool(spec.skip[l])) if l > 0 else 0
            s.W[l] = self.W[l].data_ptr()
            s.b[l] = self.b[l].data_ptr()
        amax = getattr(spec, "fp8_amax", None)
        if amax is not None:
            for l, a in enumerate(amax):
                s.fp8_amax[l] = float(a)
        self.struct = s


class DeviceCBN:
    """The conditional-batch-norm lifting network (synth.CBNSpec) on the GPU."""

    def __init__(self, spec, device="cuda"):
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device)
        self.spec = spec
        self.Wp, self.bp, self.Wo, self.bo = t(spec.Wp), t(spec.bp), t(spec.Wo), t(spec.bo)
        lists = {k: [t(a) for a in getattr(spec, k)] for k in ("W", "b", "Wg", "bg", "Wb", "bb",
                                                               "mean", "var")}
        self.lists = lists
        s = PifuCBN()
        s.feat_dim, s.n_z, s.width, s.n_blocks = spec.feat_dim, spec.n_z, spec.width, spec.n_blocks
        s.eps = spec.eps
        s.Wp, s.bp, s.Wo, s.bo = (x.data_ptr() for x in (self.Wp, self.bp, self.Wo, self.bo))
        for k, arr in lists.items():
            for i, a in enumerate(arr):
                getattr(s, k)[i] = a.data_ptr()
        self.struct = s


class DeviceField:
    """An occupancy/colour field for the C ABI (MLP over a feature map, or analytic)."""

    def __init__(self, kind: int, feat=None, mlp: Optional[DeviceMLP] = None,
                 surrogate: Optional[DeviceMLP] = None, ell=None, sharpness: float = 8.0,
                 plane=None, device="cuda"):
        s = PifuField()
        s.kind = kind
        self._keep = []
        if kind == FIELD_MLP:
            ft = torch.as_tensor(np.ascontiguousarray(feat, np.float32)).to(device) \
                if not isinstance(feat, torch.Tensor) else feat.contiguous()
            self.feat = ft
            s.H, s.W, s.C = ft.shape
            s.feat = ft.data_ptr()
            self.mlp = mlp
            s.mlp = C.pointer(mlp.struct)
            if surrogate is not None:
                s.surrogate = C.pointer(surrogate.struct)
            self.surrogate = surrogate
        elif kind == FIELD_CBN:
            ft = torch.as_tensor(np.ascontiguousarray(feat, np.float32)).to(device) \
                if not isinstance(feat, torch.Tensor) else feat.contiguous()
            self.feat = ft
            s.H, s.W, s.C = ft.shape
            s.feat = ft.data_ptr()
            self.cbn = mlp
            s.cbn = C.pointer(mlp.struct)
        elif kind == FIELD_ELLIPSOIDS:
            e = np.ascontiguousarray(ell, np.float32).reshape(-1, 12)
            self._ell = e
            s.n_ell = e.shape[0]
            s.sharpness = sharpness
            s.ell = e.ctypes.data
        elif kind == FIELD_PLANE:
            for i in range(4):
                s.plane[i] = float(plane[i])
        self.struct = s

    @staticmethod
    def mlp_field(feat, spec, surrogate_spec=None, device="cuda"):
        sur = DeviceMLP(surrogate_spec, device) if surrogate_spec is not None else None
        return DeviceField(FIELD_MLP, feat=feat, mlp=DeviceMLP(spec, device), surrogate=sur,
                           device=device)

    @staticmethod
    def cbn_field(feat, spec, device="cuda"):
        return DeviceField(FIELD_CBN, feat=feat, mlp=DeviceCBN(spec, device), device=device)

    @staticmethod
    def ellipsoids(ell, sharpness=8.0):
        return DeviceField(FIELD_ELLIPSOIDS, ell=ell, sharpness=sharpness)

    @staticmethod
    def plane_field(coef):
        return DeviceField(FIELD_PLANE, plane=coef)


# ------------------------------------------------------------------ entry points

def grid_opts(log2_final, log2_coarse, dense=False, precision="fp32", band_delta=0.02,
              guard_logit=1e-3, surrogate_max_log2=-1, surrogate_delta=0.1, tile_m=0,
              max_waves=0) -> PifuGridOpts:
    o = PifuGridOpts()
    o.log2_final, o.log2_coarse, o.dense = log2_final, log2_coarse, int(dense)
    o.precision = PREC[precision]
    o.band_delta, o.guard_logit = band_delta, guard_logit
    o.surrogate_max_log2, o.surrogate_delta = surrogate_max_log2, surrogate_delta
    o.tile_m, o.max_waves = tile_m, max_waves
    return o


def occupancy_grid_workspace_size(field: DeviceField, opts: PifuGridOpts) -> int:
    lib = load_library()
    n = C.c_size_t()
    _check(lib.pifu_occupancy_grid_workspace_size(C.byref(field.struct), C.byref(opts), C.byref(n)),
           "pifu_occupancy_grid_workspace_size")
    return n.value


class GridOutputs:
    """Preallocated outputs + workspace of pifu_occupancy_grid (reusable across calls)."""

    def __init__(self, field: DeviceField, opts: PifuGridOpts, cells_cap: Optional[int] = None,
                 eval_level: bool = False, device="cuda"):
        n = (1 << opts.log2_final) + 1
        self.opts = opts
        self.occ = torch.empty((n, n, n), dtype=torch.float32, device=device)
        self.labels = torch.empty((n, n, n), dtype=torch.uint8, device=device)
        self.eval_level = torch.empty((n, n, n), dtype=torch.uint8, device=device) if eval_level else None
        cap = cells_cap if cells_cap is not None else min((n - 1) ** 3, 1 << 26)
        self.cells = torch.empty(max(cap, 1), dtype=torch.int32, device=device)
        self.cells_cap = cap
        self.ws_bytes = occupancy_grid_workspace_size(field, opts)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        n_levels = 1 if opts.dense else opts.log2_final - opts.log2_coarse + 1
        self.stats = (PifuLevelStats * n_levels)()
        self.n_cells = C.c_uint32()


def occupancy_grid_into(field: DeviceField, out: GridOutputs, stream=None) -> None:
    lib = load_library()
    st = lib.pifu_occupancy_grid(context(), C.byref(field.struct), C.byref(out.opts),
                                 _ptr(out.occ), _ptr(out.labels), _ptr(out.eval_level),
                                 _ptr(out.cells), out.cells_cap, C.byref(out.n_cells), out.stats,
                                 _ptr(out.ws), out.ws_bytes, _stream(stream))
    _check(st, "pifu_occupancy_grid")


def occupancy_grid(field: DeviceField, log2_final: int, log2_coarse: int, *, dense=False,
                   precision="fp32", guard_logit=1e-3, band_delta=0.02, max_waves=0,
                   cells_cap=None, eval_level=False, stream=None, **kw) -> Dict[str, object]:
    """Hierarchical occupancy grid (see pifu_occupancy_grid in include/pifu.h)."""
    opts = grid_opts(log2_final, log2_coarse, dense, precision, band_delta, guard_logit,
                     max_waves=max_waves, **kw)
    out = GridOutputs(field, opts, cells_cap, eval_level)
    occupancy_grid_into(field, out, stream)
    nc = out.n_cells.value
    return dict(occ=out.occ, labels=out.labels, eval_level=out.eval_level,
                cells=out.cells[:min(nc, out.cells_cap)], n_cells=nc,
                stats=[s.as_dict() for s in out.stats])


OCTREE = {"binarized": 0, "threshold": 1}


def octree_grid_into(field: DeviceField, out: GridOutputs, mode: str, threshold: float = 0.0,
                     stream=None) -> None:
    """pifu_octree_grid into preallocated outputs (the workspace of the occupancy grid)."""
    lib = load_library()
    st = lib.pifu_octree_grid(context(), C.byref(field.struct), C.byref(out.opts), OCTREE[mode],
                              float(threshold), _ptr(out.occ), _ptr(out.labels),
                              _ptr(out.eval_level), _ptr(out.cells), out.cells_cap,
                              C.byref(out.n_cells), out.stats, _ptr(out.ws), out.ws_bytes,
                              _stream(stream))
    _check(st, "pifu_octree_grid")


def octree_grid(field: DeviceField, log2_final: int, log2_coarse: int, mode: str,
                threshold: float = 0.0, *, precision="fp32", guard_logit=1e-3, band_delta=0.02,
                cells_cap=None, eval_level=False, stream=None, **kw) -> Dict[str, object]:
    """Octree-subdivision baseline grid (see pifu_octree_grid in include/pifu.h)."""
    opts = grid_opts(log2_final, log2_coarse, False, precision, band_delta, guard_logit, **kw)
    out = GridOutputs(field, opts, cells_cap, eval_level)
    octree_grid_into(field, out, mode, threshold, stream)
    nc = out.n_cells.value
    return dict(occ=out.occ, labels=out.labels, eval_level=out.eval_level,
                cells=out.cells[:min(nc, out.cells_cap)], n_cells=nc,
                stats=[s.as_dict() for s in out.stats])


def render_opts(log2_w, log2_d, log2_coarse_w, precision="fp32", band_delta=0.02, guard_logit=1e-3,
                surrogate_max_log2=-1, surrogate_delta=0.1, tile_m=0, max_waves=0) -> PifuRenderOpts:
    o = PifuRenderOpts()
    o.log2_w, o.log2_d, o.log2_coarse_w = log2_w, log2_d, log2_coarse_w
    o.precision = PREC[precision]
    o.band_delta, o.guard_logit = band_delta, guard_logit
    o.surrogate_max_log2, o.surrogate_delta = surrogate_max_log2, surrogate_delta
    o.tile_m, o.max_waves = tile_m, max_waves
    return o


class RenderOutputs:
    def __init__(self, occ_field: DeviceField, color_field: DeviceField, opts: PifuRenderOpts,
                 device="cuda"):
        lib = load_library()
        W = 1 << opts.log2_w
        self.opts = opts
        self.rgb = torch.empty((W, W, 3), dtype=torch.float32, device=device)
        self.depth = torch.empty((W, W), dtype=torch.float32, device=device)
        self.hit = torch.empty((W, W), dtype=torch.uint8, device=device)
        n = C.c_size_t()
        _check(lib.pifu_render_view_workspace_size(C.byref(occ_field.struct),
                                                   C.byref(color_field.struct), C.byref(opts),
                                                   C.byref(n)), "pifu_render_view_workspace_size")
        self.ws_bytes = n.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.stats = (PifuLevelStats * (opts.log2_w - opts.log2_coarse_w + 1))()


def render_view_into(occ_field: DeviceField, color_field: DeviceField, view, bg,
                     out: RenderOutputs, stream=None) -> None:
    lib = load_library()
    v = (C.c_float * 12)(*[float(x) for x in np.asarray(view, np.float32).reshape(-1)])
    b = (C.c_float * 3)(*[float(x) for x in bg])
    st = lib.pifu_render_view(context(), C.byref(occ_field.struct), C.byref(color_field.struct), v,
                              C.byref(out.opts), b, _ptr(out.rgb), _ptr(out.depth), _ptr(out.hit),
                              out.stats, _ptr(out.ws), out.ws_bytes, _stream(stream))
    _check(st, "pifu_render_view")


def grid_and_render_into(field: DeviceField, gout: GridOutputs, color_field: DeviceField, view, bg,
                         rout: RenderOutputs, grid_stream=None, render_stream=None) -> None:
    """One frame (see pifu_grid_and_render in include/pifu.h): the occupancy grid on
    grid_stream and the render of `view` on render_stream, run concurrently when the
    two streams differ.  Same outputs as occupancy_grid_into + render_view_into."""
    lib = load_library()
    v = (C.c_float * 12)(*[float(x) for x in np.asarray(view, np.float32).reshape(-1)])
    b = (C.c_float * 3)(*[float(x) for x in bg])
    g = PifuGridCall(C.pointer(field.struct), C.pointer(gout.opts), _ptr(gout.occ),
                     _ptr(gout.labels), _ptr(gout.eval_level), _ptr(gout.cells), gout.cells_cap,
                     C.pointer(gout.n_cells), C.cast(gout.stats, C.POINTER(PifuLevelStats)),
                     _ptr(gout.ws), gout.ws_bytes, _stream(grid_stream))
    r = PifuRenderCall(C.pointer(field.struct), C.pointer(color_field.struct), v,
                       C.pointer(rout.opts), b, _ptr(rout.rgb), _ptr(rout.depth), _ptr(rout.hit),
                       C.cast(rout.stats, C.POINTER(PifuLevelStats)), _ptr(rout.ws),
                       rout.ws_bytes, _stream(render_stream))
    _check(lib.pifu_grid_and_render(context(), C.byref(g), C.byref(r)), "pifu_grid_and_render")


def render_view(occ_field: DeviceField, color_field: DeviceField, view, log2_w: int, log2_d: int,
                log2_coarse_w: int, bg=(0.0, 0.0, 0.0), *, precision="fp32", guard_logit=1e-3,
                band_delta=0.02, max_waves=0, stream=None, **kw) -> Dict[str, object]:
    """Mesh-free rendering of a target view (see pifu_render_view in include/pifu.h)."""
    opts = render_opts(log2_w, log2_d, log2_coarse_w, precision, band_delta, guard_logit,
                       max_waves=max_waves, **kw)
    out = RenderOutputs(occ_field, color_field, opts)
    render_view_into(occ_field, color_field, view, bg, out, stream)
    return dict(rgb=out.rgb, depth=out.depth, hit=out.hit, stats=[s.as_dict() for s in out.stats])


def render_view_traced(occ_field: DeviceField, color_field: DeviceField, view, log2_w: int,
                       log2_d: int, log2_coarse_w: int, bg=(0.0, 0.0, 0.0), *, precision="fp32",
                       guard_logit=1e-3, band_delta=0.02, max_waves=0, stream=None,
                       **kw) -> Dict[str, object]:
    """render_view plus the per-node record of pifu_render_view_traced: k* and k1 per
    pixel, and the evaluation level and logit of every node of the finest lattice."""
    lib = load_library()
    opts = render_opts(log2_w, log2_d, log2_coarse_w, precision, band_delta, guard_logit,
                       max_waves=max_waves, **kw)
    out = RenderOutputs(occ_field, color_field, opts)
    W, D = 1 << log2_w, 1 << log2_d
    kstar = torch.empty((W, W), dtype=torch.int32, device="cuda")
    k1 = torch.empty((W, W), dtype=torch.int32, device="cuda")
    evl = torch.empty((W + 1, W + 1, D + 1), dtype=torch.uint8, device="cuda")
    lg = torch.full((W + 1, W + 1, D + 1), float("nan"), dtype=torch.float32, device="cuda")
    tr = PifuRenderTrace(kstar.data_ptr(), k1.data_ptr(), evl.data_ptr(), lg.data_ptr())
    v = (C.c_float * 12)(*[float(x) for x in np.asarray(view, np.float32).reshape(-1)])
    b = (C.c_float * 3)(*[float(x) for x in bg])
    st = lib.pifu_render_view_traced(context(), C.byref(occ_field.struct),
                                     C.byref(color_field.struct), v, C.byref(out.opts), b,
                                     _ptr(out.rgb), _ptr(out.depth), _ptr(out.hit), out.stats,
                                     _ptr(out.ws), out.ws_bytes, _stream(stream), C.byref(tr))
    _check(st, "pifu_render_view_traced")
    return dict(rgb=out.rgb, depth=out.depth, hit=out.hit, stats=[s.as_dict() for s in out.stats],
                kstar=kstar, k1=k1, eval_level=evl, logit=lg)


def eval_points(field: DeviceField, pts, precision="fp32", guard_logit=1e-3, band_delta=0.02,
                stream=None, occ=False):
    """Field logits and labels at input-view NDC points (n x 3); with occ=True also the
    occupancy values p computed by the library."""
    lib = load_library()
    p = torch.as_tensor(np.asarray(pts, np.float32)) if not isinstance(pts, torch.Tensor) else pts
    n = p.shape[0]
    p4 = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    p4[:, :3] = p.to(device="cuda", dtype=torch.float32)
    logit = torch.empty(n, dtype=torch.float32, device="cuda")
    labels = torch.empty(n, dtype=torch.uint8, device="cuda")
    sz = C.c_size_t()
    _check(lib.pifu_eval_points_workspace_size(C.byref(field.struct), PREC[precision], n,
                                               C.byref(sz)), "pifu_eval_points_workspace_size")
    ws = torch.empty(sz.value, dtype=torch.uint8, device="cuda")
    p_out = torch.empty(n, dtype=torch.float32, device="cuda") if occ else None
    st = lib.pifu_eval_points(context(), C.byref(field.struct), PREC[precision], band_delta,
                              guard_logit, _ptr(p4), n, _ptr(logit), _ptr(labels), _ptr(p_out),
                              _ptr(ws), sz.value, _stream(stream))
    _check(st, "pifu_eval_points")
    return (logit, labels, p_out) if occ else (logit, labels)


def fp8_calibrate(field: DeviceField, pts, stream=None) -> List[float]:
    """Per-layer max |input| of field's network over input-view points (n x 3), from the
    library's FP32 pass: the static FP8 activation scales (pifu_mlp.fp8_amax)."""
    lib = load_library()
    p = torch.as_tensor(np.asarray(pts, np.float32)) if not isinstance(pts, torch.Tensor) else pts
    n = p.shape[0]
    p4 = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    p4[:, :3] = p.to(device="cuda", dtype=torch.float32)
    sz = C.c_size_t()
    _check(lib.pifu_eval_points_workspace_size(C.byref(field.struct), PREC["fp32"], n,
                                               C.byref(sz)), "pifu_eval_points_workspace_size")
    ws = torch.empty(sz.value, dtype=torch.uint8, device="cuda")
    nh = field.struct.mlp.contents.n_layers - 1
    out = (C.c_float * MAX_LAYERS)()
    _check(lib.pifu_fp8_calibrate(context(), C.byref(field.struct), _ptr(p4), n, out, _ptr(ws),
                                  sz.value, _stream(stream)), "pifu_fp8_calibrate")
    return [float(out[l]) for l in range(nh)]


STATS_WORDS = C.sizeof(PifuLevelStats) // 4
ASYNC_STATUS = {1: "list over max_points", 2: "waves left", 4: "guard over", 8: "cells over"}


def stats_from_device(t: torch.Tensor) -> List[Dict[str, int]]:
    """Device stats records (int32 words) -> list of dicts."""
    a = t.view(-1, STATS_WORDS).cpu()
    out = []
    for row in a:
        rec = PifuLevelStats.from_buffer_copy(bytes(row.numpy().tobytes()))
        out.append(rec.as_dict())
    return out


class AsyncGrid:
    """Outputs, device-side counts and workspace of pifu_occupancy_grid_async.  run()
    only enqueues (graph-capturable); read n_cells / stats / status after the stream."""

    def __init__(self, field: DeviceField, opts: PifuGridOpts, max_points: int = 0,
                 eval_level: bool = False, cells_cap: Optional[int] = None, device="cuda",
                 workspace: bool = True):
        """workspace=False: no workspace buffer; only run_noalloc() can be used."""
        lib = load_library()
        n = (1 << opts.log2_final) + 1
        self.field, self.opts, self.max_points = field, opts, max_points
        self.occ = torch.empty((n, n, n), dtype=torch.float32, device=device)
        self.labels = torch.empty((n, n, n), dtype=torch.uint8, device=device)
        self.eval_level = torch.empty((n, n, n), dtype=torch.uint8, device=device) if eval_level else None
        cap = cells_cap if cells_cap is not None else min((n - 1) ** 3, 1 << 26)
        self.cells = torch.empty(max(cap, 1), dtype=torch.int32, device=device)
        self.cells_cap = cap
        n_levels = 1 if opts.dense else opts.log2_final - opts.log2_coarse + 1
        self.words = torch.zeros(2 + n_levels * STATS_WORDS, dtype=torch.int32, device=device)
        sz = C.c_size_t()
        _check(lib.pifu_occupancy_grid_async_workspace_size(C.byref(field.struct), C.byref(opts),
                                                            max_points, C.byref(sz)),
               "pifu_occupancy_grid_async_workspace_size")
        self.ws_bytes = sz.value
        self.ws = torch.empty(sz.value, dtype=torch.uint8, device=device) if workspace else None

    def run_noalloc(self, stream=None):
        """pifu_occupancy_grid_async_noalloc: the same call on the library's fixed scratch."""
        p = self.words.data_ptr()
        st = load_library().pifu_occupancy_grid_async_noalloc(
            context(), C.byref(self.field.struct), C.byref(self.opts), self.max_points,
            _ptr(self.occ), _ptr(self.labels), _ptr(self.eval_level), _ptr(self.cells),
            self.cells_cap, p, p + 8, p + 4, _stream(stream))
        _check(st, "pifu_occupancy_grid_async_noalloc")

    def run(self, stream=None):
        if self.ws is None:
            raise PifuError("this AsyncGrid has no workspace: use run_noalloc()")
        p = self.words.data_ptr()
        st = load_library().pifu_occupancy_grid_async(
            context(), C.byref(self.field.struct), C.byref(self.opts), self.max_points,
            _ptr(self.occ), _ptr(self.labels), _ptr(self.eval_level), _ptr(self.cells),
            self.cells_cap, p, p + 8, p + 4, _ptr(self.ws), self.ws.numel(), _stream(stream))
        _check(st, "pifu_occupancy_grid_async")

    def result(self):
        nc = int(self.words[0].item())
        return dict(occ=self.occ, labels=self.labels, eval_level=self.eval_level,
                    cells=self.cells[:min(nc, self.cells_cap)], n_cells=nc,
                    stats=stats_from_device(self.words[2:]), status=int(self.words[1].item()))


class AsyncRender:
    """Outputs, device-side counts and workspace of pifu_render_view_async."""

    def __init__(self, occ_field: DeviceField, color_field: DeviceField, view, bg,
                 opts: PifuRenderOpts, max_points: int = 0, device="cuda"):
        lib = load_library()
        W = 1 << opts.log2_w
        self.occ_field, self.color_field, self.opts, self.max_points = occ_field, color_field, opts, max_points
        self.view = (C.c_float * 12)(*[float(x) for x in np.asarray(view, np.float32).reshape(-1)])
        self.bg = (C.c_float * 3)(*[float(x) for x in bg])
        self.rgb = torch.empty((W, W, 3), dtype=torch.float32, device=device)
        self.depth = torch.empty((W, W), dtype=torch.float32, device=device)
        self.hit = torch.empty((W, W), dtype=torch.uint8, device=device)
        n_levels = opts.log2_w - opts.log2_coarse_w + 1
        self.words = torch.zeros(2 + n_levels * STATS_WORDS, dtype=torch.int32, device=device)
        sz = C.c_size_t()
        _check(lib.pifu_render_view_async_workspace_size(C.byref(occ_field.struct),
                                                         C.byref(color_field.struct), C.byref(opts),
                                                         max_points, C.byref(sz)),
               "pifu_render_view_async_workspace_size")
        self.ws = torch.empty(sz.value, dtype=torch.uint8, device=device)

    def run(self, stream=None):
        p = self.words.data_ptr()
        st = load_library().pifu_render_view_async(
            context(), C.byref(self.occ_field.struct), C.byref(self.color_field.struct), self.view,
            C.byref(self.opts), self.max_points, self.bg, _ptr(self.rgb), _ptr(self.depth),
            _ptr(self.hit), p + 8, p + 4, _ptr(self.ws), self.ws.numel(), _stream(stream))
        _check(st, "pifu_render_view_async")

    def result(self):
        return dict(rgb=self.rgb, depth=self.depth, hit=self.hit,
                    stats=stats_from_device(self.words[2:]), status=int(self.words[1].item()))


class BatchedGrid:
    """Preallocated outputs + workspace for pifu_occupancy_grid_batched."""

    def __init__(self, fields: Sequence[DeviceField], opts: Sequence[PifuGridOpts], device="cuda"):
        lib = load_library()
        self.fields = list(fields)
        self.opts = list(opts)
        n = len(fields)
        self._f = (C.c_void_p * n)(*[C.addressof(f.struct) for f in self.fields])
        self._o = (C.c_void_p * n)(*[C.addressof(o) for o in self.opts])
        sz = C.c_size_t()
        _check(lib.pifu_occupancy_grid_batched_workspace_size(n, self._f, self._o, C.byref(sz)),
               "pifu_occupancy_grid_batched_workspace_size")
        self.ws = torch.empty(sz.value, dtype=torch.uint8, device=device)
        self.outs = (PifuGridOut * n)()
        self.occ, self.labels, self.cells, self.stats = [], [], [], []
        for i, o in enumerate(self.opts):
            m = (1 << o.log2_final) + 1
            occ = torch.empty((m, m, m), dtype=torch.float32, device=device)
            lab = torch.empty((m, m, m), dtype=torch.uint8, device=device)
            cap = min((m - 1) ** 3, 1 << 26)
            cells = torch.empty(cap, dtype=torch.int32, device=device)
            st = (PifuLevelStats * (o.log2_final - o.log2_coarse + 1))()
            self.occ.append(occ)
            self.labels.append(lab)
            self.cells.append(cells)
            self.stats.append(st)
            self.outs[i].occ = occ.data_ptr()
            self.outs[i].labels = lab.data_ptr()
            self.outs[i].cells = cells.data_ptr()
            self.outs[i].cells_cap = cap
            self.outs[i].stats = C.cast(st, C.POINTER(PifuLevelStats))

    def run(self, stream=None):
        lib = load_library()
        st = lib.pifu_occupancy_grid_batched(context(), len(self.fields), self._f, self._o,
                                             self.outs, self.ws.data_ptr(), self.ws.numel(),
                                             _stream(stream))
        _check(st, "pifu_occupancy_grid_batched")

    def result(self, i):
        nc = self.outs[i].n_cells
        return dict(occ=self.occ[i], labels=self.labels[i],
                    cells=self.cells[i][:min(nc, self.outs[i].cells_cap)], n_cells=nc,
                    stats=[s.as_dict() for s in self.stats[i]])


class AsyncBatchedGrid:
    """Outputs, device-side counts and workspace of pifu_occupancy_grid_batched_async.
    run() only enqueues (graph-capturable); read results after the stream."""

    def __init__(self, fields: Sequence[DeviceField], opts: Sequence[PifuGridOpts],
                 max_points: int = 0, device="cuda"):
        lib = load_library()
        self.fields = list(fields)
        self.opts = list(opts)
        self.max_points = max_points
        n = len(fields)
        self._f = (C.c_void_p * n)(*[C.addressof(f.struct) for f in self.fields])
        self._o = (C.c_void_p * n)(*[C.addressof(o) for o in self.opts])
        sz = C.c_size_t()
        _check(lib.pifu_occupancy_grid_batched_async_workspace_size(n, self._f, self._o,
                                                                    max_points, C.byref(sz)),
               "pifu_occupancy_grid_batched_async_workspace_size")
        self.ws = torch.empty(sz.value, dtype=torch.uint8, device=device)
        self.outs = (PifuGridOutDev * n)()
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.occ, self.labels, self.cells, self.words = [], [], [], []
        for i, o in enumerate(self.opts):
            m = (1 << o.log2_final) + 1
            occ = torch.empty((m, m, m), dtype=torch.float32, device=device)
            lab = torch.empty((m, m, m), dtype=torch.uint8, device=device)
            cap = min((m - 1) ** 3, 1 << 26)
            cells = torch.empty(cap, dtype=torch.int32, device=device)
            nlev = o.log2_final - o.log2_coarse + 1
            words = torch.zeros(1 + nlev * STATS_WORDS, dtype=torch.int32, device=device)
            self.occ.append(occ)
            self.labels.append(lab)
            self.cells.append(cells)
            self.words.append(words)
            self.outs[i].occ = occ.data_ptr()
            self.outs[i].labels = lab.data_ptr()
            self.outs[i].cells = cells.data_ptr()
            self.outs[i].cells_cap = cap
            self.outs[i].n_cells_dev = words.data_ptr()
            self.outs[i].stats_dev = words.data_ptr() + 4

    def run(self, stream=None):
        st = load_library().pifu_occupancy_grid_batched_async(
            context(), len(self.fields), self._f, self._o, self.max_points, self.outs,
            self.status.data_ptr(), self.ws.data_ptr(), self.ws.numel(), _stream(stream))
        _check(st, "pifu_occupancy_grid_batched_async")

    def result(self, i):
        nc = int(self.words[i][0].item())
        return dict(occ=self.occ[i], labels=self.labels[i],
                    cells=self.cells[i][:min(nc, self.outs[i].cells_cap)], n_cells=nc,
                    stats=stats_from_device(self.words[i][1:]),
                    status=int(self.status[0].item()))


class OhemSampler:
    """Point-OHEM (Sec. 3.3, Eq. 6 right) over a pool of training points: stored inverse
    probabilities (initially 1), weighted draws (pifu_ohem_sample) and the update from
    per-point losses (pifu_ohem_update)."""

    def __init__(self, pool: torch.Tensor, batch: int, seed: int = 0, alpha: float = 0.7,
                 beta: float = 0.0):
        lib = load_library()
        assert pool.dtype == torch.float32 and pool.shape[1] == 4 and pool.is_contiguous()
        self.pool, self.batch, self.seed = pool, batch, seed
        self.alpha, self.beta = alpha, beta
        n = pool.shape[0]
        self.weights = torch.ones(n, dtype=torch.float32, device=pool.device)
        self.idx = torch.empty(batch, dtype=torch.int32, device=pool.device)
        self.pts = torch.empty((batch, 4), dtype=torch.float32, device=pool.device)
        sz = C.c_size_t()
        _check(lib.pifu_ohem_sample_workspace_size(n, C.byref(sz)), "pifu_ohem_sample_workspace_size")
        self.ws = torch.empty(sz.value, dtype=torch.uint8, device=pool.device)
        self.counter = 0

    def draw(self, stream=None) -> torch.Tensor:
        st = load_library().pifu_ohem_sample(
            context(), self.weights.data_ptr(), self.pool.shape[0], self.pool.data_ptr(),
            self.batch, self.seed, self.counter, self.idx.data_ptr(), self.pts.data_ptr(),
            self.ws.data_ptr(), self.ws.numel(), _stream(stream))
        _check(st, "pifu_ohem_sample")
        self.counter += 1
        return self.pts

    def update(self, point_loss: torch.Tensor, stream=None) -> None:
        st = load_library().pifu_ohem_update(context(), point_loss.data_ptr(), self.idx.data_ptr(),
                                             self.batch, self.alpha, self.beta,
                                             self.weights.data_ptr(), _stream(stream))
        _check(st, "pifu_ohem_update")


def mesh(occ: torch.Tensor, labels: torch.Tensor, cells: torch.Tensor,
         color_field: Optional[DeviceField] = None, image: Optional[torch.Tensor] = None,
         vert_cap: Optional[int] = None, tri_cap: Optional[int] = None,
         stream=None) -> Dict[str, object]:
    """Marching Cubes over the surface cells (pifu_mesh): vertices, triangles and, with a
    colour field, vertex colours (the input pixel where visible when an image is given)."""
    lib = load_library()
    n = occ.shape[0]
    L = (n - 1).bit_length() - 1
    nc = int(cells.numel())
    vcap = vert_cap if vert_cap is not None else max(4 * nc, 16)
    tcap = tri_cap if tri_cap is not None else max(5 * nc, 16)
    fs = C.byref(color_field.struct) if color_field is not None else None
    sz = C.c_size_t()
    _check(lib.pifu_mesh_workspace_size(L, nc, vcap, fs, C.byref(sz)), "pifu_mesh_workspace_size")
    ws = torch.empty(sz.value, dtype=torch.uint8, device=occ.device)
    verts = torch.empty((vcap, 3), dtype=torch.float32, device=occ.device)
    colors = torch.empty((vcap, 3), dtype=torch.float32, device=occ.device) if color_field is not None else None
    tris = torch.empty((tcap, 3), dtype=torch.int32, device=occ.device)
    nv, nt = C.c_uint32(), C.c_uint32()
    img = image.contiguous() if image is not None else None
    st = lib.pifu_mesh(context(), L, occ.data_ptr(), labels.data_ptr(),
                       cells.data_ptr() if nc else None, nc, fs, _ptr(img),
                       img.shape[0] if img is not None else 0, img.shape[1] if img is not None else 0,
                       verts.data_ptr(), _ptr(colors), vcap, C.byref(nv), tris.data_ptr(), tcap,
                       C.byref(nt), ws.data_ptr(), ws.numel(), _stream(stream))
    _check(st, "pifu_mesh")
    v, t = nv.value, nt.value
    return dict(verts=verts[:min(v, vcap)], colors=colors[:min(v, vcap)] if colors is not None else None,
                tris=tris[:min(t, tcap)], n_verts=v, n_tris=t)
