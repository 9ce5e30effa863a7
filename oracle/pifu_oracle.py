"""Plain FP64 CPU oracle for hierarchical surface localization and mesh-free rendering.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library; the only common module is ``synth`` (seeded inputs).

Paper: Li et al., "Monocular Real-Time Volumetric Performance Capture", ECCV 2020.
  * Eq. 1 (Sec. 3.1): O(P) = f_O(Phi(P_xy, g_O(I)), P_z), surface = 0.5 level set.
  * Sec. 3.2, "Octree-based Robust Surface Localization": binarize the coarser
    level at 0.5, trilinearly interpolate to the current level, take the nodes
    whose value is neither 0 nor 1, dilate by the 1-ring, evaluate, then
    evaluate neighbours of conflict nodes until no conflict is left.
  * Sec. 3.2, "Mesh-free Rendering" and Eq. 3: localize to level L-1 on the
    target-view grid, upsample + argmax along z, shadow nodes, evaluate the
    rest, argmax again, interpolate the surface point, colour it with Eq. 2.

Readings of the paper where it is silent or ambiguous (kept identical on the GPU):
  * a grid of "2^L" has 2^L cells, i.e. 2^L + 1 nodes per axis; node i sits at
    NDC -1 + 2 i / 2^L; coarse nodes are the even fine nodes.
  * pixel coordinates u = (x+1)/2 (W-1), v = (y+1)/2 (H-1); texels outside the
    map contribute 0 to the bilinear sum.
  * label = [logit > 0]; p = sigmoid(logit) is the occupancy value.
  * dilation and "adjacent" use the 26-neighbourhood on the level's lattice.
  * the conflict test compares [logit > 0] with [interp > 1/2]; conflict waves
    are synchronous and stop when a wave adds no node.
  * render rays run from the observer (z = +1, largest k) inwards; no conflict
    loop at the last render level; points outside the input volume after the
    view transform have logit -inf.
  * the surface point is the 0.5 crossing of the linear interpolation of the
    two nodes' occupancy values along z.
  * the octree baselines compared in Sec. 3.2 / Fig. 3 subdivide the closed 3x3x3 node
    blocks of the selected coarse cells, with no dilation and no conflict search.
  * point-OHEM (Sec. 3.3, Eq. 6 right) caps the inverse probability at 2^20 and draws
    with integer-quantised weights and the SplitMix64 generator.
  * the mesh hand-off (Marching Cubes) derives its 256-case table from the contour on the
    cube faces; conventions are listed with the mesh functions below.

Parity: every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` (closed forms, library routines, invariants, brute
force on tiny grids).  The paper prints no worked example of the algorithm.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

# ------------------------------------------------------------------ evaluate

LRELU_SLOPE = 0.01


def sigmoid(logit: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-logit))


def bilinear_sample(F: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Phi(P_xy, F): bilinear sampling of an HWC feature map at NDC (x, y) (Eq. 1).

    Column u runs along x and row v along y.  Texels outside the map count as 0.
    """
    H, W, C = F.shape
    F = np.asarray(F, np.float64)
    u = (x + 1.0) * 0.5 * (W - 1)
    v = (y + 1.0) * 0.5 * (H - 1)
    u0 = np.floor(u)
    v0 = np.floor(v)
    fu = u - u0
    fv = v - v0
    out = np.zeros((x.shape[0], C))
    for du, dv, w in ((0, 0, (1 - fu) * (1 - fv)), (1, 0, fu * (1 - fv)),
                      (0, 1, (1 - fu) * fv), (1, 1, fu * fv)):
        uu = (u0 + du).astype(np.int64)
        vv = (v0 + dv).astype(np.int64)
        inside = (uu >= 0) & (uu <= W - 1) & (vv >= 0) & (vv <= H - 1)
        tex = F[np.clip(vv, 0, H - 1), np.clip(uu, 0, W - 1), :]
        out += (w * inside)[:, None] * tex
    return out


def _act(h: np.ndarray, kind: str) -> np.ndarray:
    if kind == "relu":
        return np.maximum(h, 0.0)
    if kind == "lrelu":
        return np.where(h > 0, h, LRELU_SLOPE * h)
    raise ValueError(kind)


def mlp_preact(spec, f: np.ndarray, extras: np.ndarray) -> np.ndarray:
    """Output pre-activation of the MLP f_O / f_T for point features f and extras.

    Layer 0 reads [f; extras] (extras = z, or z and occ for the colour network,
    Eq. 1 / Eq. 2); hidden layer l reads [h_{l-1}; f] where the spec has a skip.
    """
    f = np.asarray(f, np.float64)
    x = np.concatenate([f, np.asarray(extras, np.float64).reshape(f.shape[0], -1)], axis=1)
    n_layers = len(spec.widths)
    h = x
    for l in range(n_layers):
        if l > 0 and spec.skip[l]:
            h = np.concatenate([h, f], axis=1)
        h = h @ np.asarray(spec.W[l], np.float64).T + np.asarray(spec.b[l], np.float64)
        if l < n_layers - 1:
            h = _act(h, spec.hidden_act)
    return h


@dataclass
class Field:
    """An occupancy field: an MLP over a feature map (Eq. 1) or an analytic stand-in."""
    kind: str                              # "mlp" | "cbn" | "ellipsoids" | "plane"
    feat: Optional[np.ndarray] = None      # H x W x C
    mlp: object = None                     # synth.MLPSpec, or synth.CBNSpec for "cbn"
    ell: Optional[np.ndarray] = None       # n x 12
    sharpness: float = 8.0
    plane: Optional[np.ndarray] = None     # a, b, c, d


def field_logit(fld: Field, P: np.ndarray, chunk: int = 32768) -> np.ndarray:
    """logit of O(P) at input-view NDC points P (n x 3)."""
    P = np.asarray(P, np.float64)
    n = P.shape[0]
    if fld.kind == "plane":
        a = np.asarray(fld.plane, np.float64)
        return P @ a[:3] + a[3]
    if fld.kind == "ellipsoids":
        E = np.asarray(fld.ell, np.float64)
        qmin = np.full(n, np.inf)
        for e in range(E.shape[0]):
            c = E[e, :3]
            M = E[e, 3:].reshape(3, 3)
            d = (P - c) @ M.T
            qmin = np.minimum(qmin, np.sum(d * d, axis=1))
        return fld.sharpness * (1.0 - qmin)
    if fld.kind == "mlp":
        out = np.empty(n)
        for s in range(0, n, chunk):
            Pc = P[s:s + chunk]
            f = bilinear_sample(fld.feat, Pc[:, 0], Pc[:, 1])
            out[s:s + chunk] = mlp_preact(fld.mlp, f, Pc[:, 2:3])[:, 0]
        return out
    if fld.kind == "cbn":
        out = np.empty(n)
        for s in range(0, n, chunk):
            Pc = P[s:s + chunk]
            f = bilinear_sample(fld.feat, Pc[:, 0], Pc[:, 1])
            out[s:s + chunk] = cbn_logit(fld.mlp, f, Pc[:, 2])
        return out
    raise ValueError(fld.kind)


def apply_view(view: np.ndarray, P: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """P' = A P + t for a 3x4 row-major view; also the mask P' in [-1,1]^3."""
    V = np.asarray(view, np.float64).reshape(3, 4)
    P = np.asarray(P, np.float64)
    Pp = np.empty_like(P)
    for r in range(3):   # elementwise, fixed order, no fused multiply-add
        Pp[:, r] = ((V[r, 0] * P[:, 0] + V[r, 1] * P[:, 1]) + V[r, 2] * P[:, 2]) + V[r, 3]
    inside = np.all((Pp >= -1.0) & (Pp <= 1.0), axis=1)
    return Pp, inside


def view_logit(fld: Field, view: Optional[np.ndarray], P: np.ndarray) -> np.ndarray:
    """Evaluate a target-view point: transform into the input view; outside -> -inf."""
    if view is None:
        return field_logit(fld, P)
    Pp, inside = apply_view(view, P)
    out = np.full(P.shape[0], -np.inf)
    if inside.any():
        out[inside] = field_logit(fld, Pp[inside])
    return out


# ------------------------------------------------------------------ grids

def lattice_coords(dims: Tuple[int, int, int], flat_idx: np.ndarray) -> np.ndarray:
    """NDC coordinates of level-lattice nodes given by linear index (z fastest)."""
    nx, ny, nz = dims
    i = flat_idx // (ny * nz)
    j = (flat_idx // nz) % ny
    k = flat_idx % nz
    return np.stack([-1.0 + 2.0 * i / (nx - 1), -1.0 + 2.0 * j / (ny - 1),
                     -1.0 + 2.0 * k / (nz - 1)], axis=1)


def upsample_x2(coarse: np.ndarray) -> np.ndarray:
    """Trilinear interpolation of a node array onto the lattice with half the spacing.

    Fine node 2a keeps coarse node a; fine node 2a+1 takes the mean of coarse nodes
    a and a+1 -- along each axis in turn, which is trilinear interpolation
    of the node values (Sec. 3.2, the interpolation step of the localization).
    """
    out = np.asarray(coarse, np.float64)
    for ax in range(3):
        n = out.shape[ax]
        shape = list(out.shape)
        shape[ax] = 2 * n - 1
        fine = np.empty(shape)
        even = [slice(None)] * 3
        odd = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        even[ax] = slice(0, None, 2)
        odd[ax] = slice(1, None, 2)
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        fine[tuple(even)] = out
        fine[tuple(odd)] = 0.5 * (out[tuple(lo)] + out[tuple(hi)])
        out = fine
    return out


def neighbourhood26(mask: np.ndarray) -> np.ndarray:
    """Nodes whose index differs from a marked node by at most 1 along every axis.

    This is the 1-ring (26-neighbourhood) dilation of Sec. 3.2, clipped at the
    grid edge; the marked nodes themselves are included.
    """
    out = np.zeros_like(mask, dtype=bool)
    pts = np.argwhere(mask)
    if pts.size == 0:
        return out
    dims = np.array(mask.shape)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for dk in (-1, 0, 1):
                q = pts + np.array([di, dj, dk])
                ok = np.all((q >= 0) & (q < dims), axis=1)
                q = q[ok]
                out[q[:, 0], q[:, 1], q[:, 2]] = True
    return out


@dataclass
class LevelRecord:
    level: int                 # log2 of the x cell count at this level
    dims: Tuple[int, int, int]
    evaluated: np.ndarray      # sorted linear indices (level lattice) evaluated at this level
    stats: Dict[str, int]


@dataclass
class LocalizeResult:
    dims: Tuple[int, int, int]          # lattice of the last level run
    val: np.ndarray                     # occupancy value: p if evaluated, else interp (0/1)
    label: np.ndarray                   # uint8 0/1
    logit: np.ndarray                   # logit where evaluated, nan elsewhere
    evaluated: np.ndarray               # bool, evaluated at any level
    levels: List[LevelRecord] = dc_field(default_factory=list)


def _eval_mask(evaluate, dims, mask):
    idx = np.flatnonzero(mask.reshape(-1))
    logit = evaluate(lattice_coords(dims, idx)) if idx.size else np.zeros(0)
    return idx, logit


def localize(evaluate: Callable[[np.ndarray], np.ndarray], log2_cells: Tuple[int, int, int],
             n_refine: int, last_level: Optional[int] = None,
             max_waves: int = 1 << 30) -> LocalizeResult:
    """Coarse-to-fine surface localization (Sec. 3.2, "Octree-based Robust Surface
    Localization").

    ``log2_cells`` are the per-axis log2 cell counts of the finest lattice and
    ``n_refine`` the number of x2 refinements above the coarsest level, which is
    evaluated densely.  Runs levels 0..last_level (default n_refine).
    """
    T = n_refine
    last = T if last_level is None else last_level
    dims_at = lambda t: tuple((1 << (L - (T - t))) + 1 for L in log2_cells)
    level_id = lambda t: log2_cells[0] - (T - t)

    # coarsest level: every node is evaluated
    dims = dims_at(0)
    allmask = np.ones(dims, bool)
    idx, logit_e = _eval_mask(evaluate, dims, allmask)
    logit = logit_e.reshape(dims)
    label = (logit > 0).astype(np.uint8)
    val = sigmoid(logit)
    evaluated = allmask.copy()
    res_levels = [LevelRecord(level_id(0), dims, idx, dict(
        nodes=int(np.prod(dims)), b0=0, dilated=int(idx.size), evaluated=int(idx.size),
        waves=0, conflicts=0))]

    for t in range(1, last + 1):
        fdims = dims_at(t)
        # binarize the coarser level at 0.5 and interpolate to this level
        interp = upsample_x2(label.astype(np.float64))
        assert interp.shape == fdims
        coarse_pos = np.zeros(fdims, bool)
        coarse_pos[::2, ::2, ::2] = True
        f_eval = np.zeros(fdims, bool)
        f_eval[::2, ::2, ::2] = evaluated
        f_val = interp.copy()
        f_val[::2, ::2, ::2] = val
        f_logit = np.full(fdims, np.nan)
        f_logit[::2, ::2, ::2] = logit
        f_label = (interp > 0.5).astype(np.uint8)     # culled nodes: interp is 0 or 1
        f_label[::2, ::2, ::2] = label
        # boundary candidates: neither 0 nor 1; then the 1-ring dilation
        b0 = (interp > 0.0) & (interp < 1.0)
        cand = neighbourhood26(b0) & ~f_eval
        now = np.zeros(fdims, bool)
        interp_hi = interp > 0.5

        def run(mask):
            idx_, lg = _eval_mask(evaluate, fdims, mask)
            flat_l = f_logit.reshape(-1)
            flat_l[idx_] = lg
            f_label.reshape(-1)[idx_] = (lg > 0).astype(np.uint8)
            f_val.reshape(-1)[idx_] = sigmoid(lg)
            f_eval.reshape(-1)[idx_] = True
            now.reshape(-1)[idx_] = True
            # conflict: network label differs from the binarized interpolation
            return mask & ((f_label == 1) != interp_hi)

        n_dilated = int(cand.sum())
        conflict = run(cand)
        n_conf = int(conflict.sum())
        waves = 0
        while conflict.any() and waves < max_waves:
            nxt = neighbourhood26(conflict) & ~f_eval
            if not nxt.any():
                break
            waves += 1
            conflict = run(nxt)
            n_conf += int(conflict.sum())
        logit, label, val, evaluated = f_logit, f_label, f_val, f_eval
        res_levels.append(LevelRecord(level_id(t), fdims, np.flatnonzero(now.reshape(-1)), dict(
            nodes=int(np.prod(fdims)), b0=int(b0.sum()), dilated=n_dilated,
            evaluated=int(now.sum()), waves=waves, conflicts=n_conf)))
        dims = fdims
    return LocalizeResult(dims, val, label, logit, evaluated, res_levels)


# ------------------------------------------------------------------ octree baselines

def _cells_of_nodes(flag: np.ndarray, fdims) -> np.ndarray:
    """Fine-lattice nodes that lie in (inside or on the boundary of) a flagged coarse cell.

    Coarse cell (a, b, c) spans fine nodes 2a..2a+2 along each axis; ``flag`` has one
    entry per coarse cell."""
    out = np.zeros(fdims, bool)
    for a, b, c in np.argwhere(flag):
        out[2 * a:2 * a + 3, 2 * b:2 * b + 3, 2 * c:2 * c + 3] = True
    return out


def _corner_stack(v: np.ndarray) -> List[np.ndarray]:
    """The 8 corner values of every cell of a node array (cells (n-1)^3)."""
    return [v[di:v.shape[0] - 1 + di, dj:v.shape[1] - 1 + dj, dk:v.shape[2] - 1 + dk]
            for di in (0, 1) for dj in (0, 1) for dk in (0, 1)]


def octree_step(val: np.ndarray, label: np.ndarray, evaluated: np.ndarray, mode: str,
                thr: float = 0.0):
    """One level of the octree subdivision (see octree_localize): from a level's node
    values, labels and evaluated flags, the cells it subdivides, the finer level's
    interpolated values and labels (before any evaluation) and the finer nodes to
    evaluate.  Returns (flag per coarse cell, f_val, f_label, f_eval, todo)."""
    fdims = tuple(2 * n - 1 for n in val.shape)
    if mode == "binarized":
        corners = _corner_stack(label.astype(bool))
        anyv = np.zeros_like(corners[0])
        allv = np.ones_like(corners[0])
        for c in corners:
            anyv |= c
            allv &= c
        flag = anyv & ~allv
        interp = upsample_x2(label.astype(np.float64))
    else:
        corners = _corner_stack(val)
        mean = sum(corners) / 8.0
        dev = np.zeros_like(mean)
        for c in corners:
            dev = np.maximum(dev, np.abs(c - mean))
        flag = dev > thr
        interp = upsample_x2(val)
    f_eval = np.zeros(fdims, bool)
    f_eval[::2, ::2, ::2] = evaluated
    f_val = interp.copy()
    f_val[::2, ::2, ::2] = val
    f_label = (interp > 0.5).astype(np.uint8)
    f_label[::2, ::2, ::2] = label
    todo = _cells_of_nodes(flag, fdims) & ~f_eval
    return flag, f_val, f_label, f_eval, todo


def octree_localize(evaluate: Callable[[np.ndarray], np.ndarray], log2_cells: Tuple[int, int, int],
                    n_refine: int, mode: str, thr: float = 0.0) -> LocalizeResult:
    """The two octree subdivisions the paper compares its localization with (Sec. 3.2,
    "Octree-based Robust Surface Localization", and the Fig. 3 comparison).

    From the densely evaluated coarsest level, each level subdivides the coarse cells
    selected by a rule and evaluates every node of those cells that was not evaluated
    before; there is no dilation and no conflict search.
      * mode "binarized": a cell is subdivided when the binarized occupancy [p > 0.5] of
        its 8 corners is not all equal (the interface between inside and outside nodes).
        Nodes of other cells take the trilinear interpolation of the binarized corner
        labels (0 or 1 there).
      * mode "threshold": a cell is subdivided when the maximum absolute deviation of
        its 8 corner occupancy values from their mean exceeds thr.  Nodes of other cells
        take the trilinear interpolation of the corner occupancy values; their label is
        [value > 0.5].
    Values are float64 occupancies p = sigmoid(logit).
    """
    assert mode in ("binarized", "threshold")
    T = n_refine
    dims_at = lambda t: tuple((1 << (L - (T - t))) + 1 for L in log2_cells)
    level_id = lambda t: log2_cells[0] - (T - t)
    dims = dims_at(0)
    idx, lg = _eval_mask(evaluate, dims, np.ones(dims, bool))
    logit = lg.reshape(dims)
    label = (logit > 0).astype(np.uint8)
    val = sigmoid(logit)
    evaluated = np.ones(dims, bool)
    levels = [LevelRecord(level_id(0), dims, idx, dict(nodes=int(np.prod(dims)),
                                                       evaluated=int(idx.size), subdivided=0))]
    for t in range(1, T + 1):
        fdims = dims_at(t)
        flag, f_val, f_label, f_eval, todo = octree_step(val, label, evaluated, mode, thr)
        f_logit = np.full(fdims, np.nan)
        f_logit[::2, ::2, ::2] = logit
        idx, lg = _eval_mask(evaluate, fdims, todo)
        f_logit.reshape(-1)[idx] = lg
        f_label.reshape(-1)[idx] = (lg > 0).astype(np.uint8)
        f_val.reshape(-1)[idx] = sigmoid(lg)
        f_eval.reshape(-1)[idx] = True
        logit, label, val, evaluated = f_logit, f_label, f_val, f_eval
        levels.append(LevelRecord(level_id(t), fdims, idx, dict(
            nodes=int(np.prod(fdims)), evaluated=int(idx.size), subdivided=int(flag.sum()))))
    return LocalizeResult(dims_at(T), val, label, logit, evaluated, levels)


def octree_grid(fld: Field, log2_final: int, log2_coarse: int, mode: str,
                thr: float = 0.0) -> Dict[str, object]:
    """Octree-subdivision occupancy grid of the input view (see octree_localize)."""
    res = octree_localize(lambda P: field_logit(fld, P), (log2_final,) * 3,
                          log2_final - log2_coarse, mode, thr)
    return dict(occ=res.val, labels=res.label, logit=res.logit, cells=surface_cells(res.label),
                eval_level=eval_level_map(res), levels=res.levels, result=res)


def surface_cells(label: np.ndarray) -> np.ndarray:
    """Sorted linear indices (i*Ry + j)*Rz + k of cells whose 8 corner labels differ."""
    L = label.astype(bool)
    corners = [L[di:L.shape[0] - 1 + di, dj:L.shape[1] - 1 + dj, dk:L.shape[2] - 1 + dk]
               for di in (0, 1) for dj in (0, 1) for dk in (0, 1)]
    anyv = np.zeros_like(corners[0])
    allv = np.ones_like(corners[0])
    for c in corners:
        anyv |= c
        allv &= c
    return np.flatnonzero((anyv & ~allv).reshape(-1)).astype(np.uint32)


def eval_level_map(res: LocalizeResult) -> np.ndarray:
    """Per finest-lattice node: level id at which it was evaluated, 255 if never."""
    out = np.full(res.dims, 255, np.uint8)
    T = len(res.levels) - 1
    for t, rec in enumerate(res.levels):
        s = 1 << (T - t)
        m = np.zeros(rec.dims, bool).reshape(-1)
        m[rec.evaluated] = True
        m = m.reshape(rec.dims)
        sub = out[::s, ::s, ::s]
        sub[m] = rec.level
    return out


def occupancy_grid(fld: Field, log2_final: int, log2_coarse: int,
                   max_waves: int = 1 << 30) -> Dict[str, object]:
    """Hierarchical occupancy grid of the input view, 2^L cells per axis."""
    res = localize(lambda P: field_logit(fld, P), (log2_final,) * 3, log2_final - log2_coarse,
                   max_waves=max_waves)
    return dict(occ=res.val, labels=res.label, logit=res.logit, cells=surface_cells(res.label),
                eval_level=eval_level_map(res), levels=res.levels, result=res)


def dense_grid(fld: Field, log2_final: int) -> Dict[str, object]:
    """Brute-force baseline: evaluate every node of the final grid."""
    n = (1 << log2_final) + 1
    dims = (n, n, n)
    logit = field_logit(fld, lattice_coords(dims, np.arange(n ** 3))).reshape(dims)
    label = (logit > 0).astype(np.uint8)
    return dict(occ=sigmoid(logit), labels=label, logit=logit, cells=surface_cells(label))


# ------------------------------------------------------------------ render

def render_view(occ_fld: Field, color_fld: Optional[Field], view: np.ndarray, log2_w: int,
                log2_d: int, log2_coarse_w: int, bg=(0.0, 0.0, 0.0),
                evaluate: Optional[Callable[[np.ndarray], np.ndarray]] = None) -> Dict[str, object]:
    """Mesh-free rendering (Sec. 3.2 and Eq. 3) on the target-view lattice.

    The lattice has W+1 x H+1 x D+1 nodes (W = H = 2^log2_w, D = 2^log2_d); pixel
    (v, u) of the W x H image is node column (u, v).  Rays run from k = D (nearest
    the observer) to k = 0.  ``evaluate`` (optional) replaces the occupancy field's
    logit at target-lattice points (a replay of recorded values); without a colour
    field the hits are not coloured.
    """
    T = log2_w - log2_coarse_w
    Wd = 1 << log2_w
    D = 1 << log2_d
    if evaluate is None:
        evaluate = lambda P: view_logit(occ_fld, view, P)
    loc = localize(evaluate, (log2_w, log2_w, log2_d), T, last_level=T - 1)
    lab_c = loc.label
    # level L: upsample the binarized labels of level L-1
    interp = upsample_x2(lab_c.astype(np.float64))[:Wd, :Wd, :]
    cur = interp.copy()
    lab = interp.copy()
    evald = np.zeros(interp.shape, bool)
    sub_v = loc.val[: Wd // 2, : Wd // 2, :]
    cur[::2, ::2, ::2] = sub_v
    lab[::2, ::2, ::2] = lab_c[: Wd // 2, : Wd // 2, :]
    evald[::2, ::2, ::2] = loc.evaluated[: Wd // 2, : Wd // 2, :]
    # argmax along z from the observer: first node with interpolated value 1
    is_one = interp == 1.0
    kk = np.arange(D + 1)
    kstar = np.where(is_one.any(axis=2), np.max(np.where(is_one, kk, -1), axis=2), -1)
    shadow = kk[None, None, :] < kstar[:, :, None]
    todo = (~shadow) & (interp > 0.0) & (interp < 1.0) & ~evald
    idx = np.flatnonzero(todo.reshape(-1))
    dims_L = (Wd + 1, Wd + 1, D + 1)
    # linear index in the full level-L lattice for coordinates
    ii = idx // ((Wd) * (D + 1))
    jj = (idx // (D + 1)) % Wd
    k_ = idx % (D + 1)
    full_idx = (ii * dims_L[1] + jj) * dims_L[2] + k_
    lg = evaluate(lattice_coords(dims_L, full_idx)) if idx.size else np.zeros(0)
    cur.reshape(-1)[idx] = sigmoid(lg)
    lab.reshape(-1)[idx] = (lg > 0).astype(np.float64)
    # binarize and argmax again
    is_in = lab == 1.0
    k1 = np.where(is_in.any(axis=2), np.max(np.where(is_in, kk, -1), axis=2), -1)
    hit = k1 >= 0
    zk = -1.0 + 2.0 * kk / D
    depth = np.full((Wd, Wd), np.nan)      # indexed [u, v] here, transposed on return
    occ_hit = np.zeros((Wd, Wd))
    us, vs = np.nonzero(hit)
    for u, v in zip(us, vs):
        k = k1[u, v]
        if k == D:
            z = 1.0
        else:
            o_f = cur[u, v, k + 1]
            o_b = cur[u, v, k]
            t = (0.5 - o_f) / (o_b - o_f) if o_b - o_f > 0 else 0.0
            z = zk[k + 1] + t * (zk[k] - zk[k + 1])
        depth[u, v] = z
        occ_hit[u, v] = cur[u, v, k]
    rgb = np.empty((Wd, Wd, 3))
    rgb[:] = np.asarray(bg, np.float64)
    if us.size and color_fld is not None:
        xs = -1.0 + 2.0 * us / Wd
        ys = -1.0 + 2.0 * vs / Wd
        P = np.stack([xs, ys, depth[us, vs]], axis=1)
        Pp, _ = apply_view(view, P)
        f = bilinear_sample(color_fld.feat, Pp[:, 0], Pp[:, 1])
        pre = mlp_preact(color_fld.mlp, f, np.stack([Pp[:, 2], occ_hit[us, vs]], axis=1))
        rgb[us, vs] = np.tanh(pre)
    stats = dict(shadow=int(shadow.sum()), evaluated_last=int(idx.size), hits=int(hit.sum()))
    return dict(rgb=np.transpose(rgb, (1, 0, 2)), depth=depth.T, hit=hit.T.astype(np.uint8),
                kstar=kstar.T, k1=k1.T, levels=loc.levels, last_eval=idx, loc=loc, stats=stats,
                eval_mask_last=todo)


# ------------------------------------------------------------------ surrogate training

def mlp_forward_cache(spec, f: np.ndarray, extras: np.ndarray):
    """Forward pass keeping every layer input and pre-activation (for the backward pass)."""
    f = np.asarray(f, np.float64)
    x0 = np.concatenate([f, np.asarray(extras, np.float64).reshape(f.shape[0], -1)], axis=1)
    ins, pres = [], []
    h = x0
    n = len(spec.widths)
    for l in range(n):
        if l > 0 and spec.skip[l]:
            h = np.concatenate([h, f], axis=1)
        ins.append(h)
        z = h @ np.asarray(spec.W[l], np.float64).T + np.asarray(spec.b[l], np.float64)
        pres.append(z)
        h = _act(z, spec.hidden_act) if l < n - 1 else z
    return ins, pres


def bce_soft(s: np.ndarray, target: np.ndarray) -> Tuple[float, np.ndarray]:
    """Binary cross entropy with soft targets on logits s (the loss the paper uses for
    occupancy, Sec. 3.1), mean over the batch.  Returns (loss, dloss/ds)."""
    s = np.asarray(s, np.float64)
    t = np.asarray(target, np.float64)
    loss_each = np.logaddexp(0.0, s) - t * s     # softplus(s) - t s
    return float(loss_each.mean()), (sigmoid(s) - t) / s.shape[0]


def mlp_backward(spec, ins, pres, dout: np.ndarray):
    """Weight and bias gradients of the MLP given dloss/d(output pre-activation)."""
    n = len(spec.widths)
    dW = [None] * n
    db = [None] * n
    g = np.asarray(dout, np.float64).reshape(pres[-1].shape)
    for l in range(n - 1, -1, -1):
        dW[l] = g.T @ ins[l]
        db[l] = g.sum(axis=0)
        if l == 0:
            break
        dx = g @ np.asarray(spec.W[l], np.float64)
        dh = dx[:, : spec.widths[l - 1]]
        if spec.hidden_act == "relu":
            g = dh * (pres[l - 1] > 0)
        else:
            g = dh * np.where(pres[l - 1] > 0, 1.0, LRELU_SLOPE)
    return dW, db


def rmsprop_step(w: np.ndarray, g: np.ndarray, v: np.ndarray, lr: float = 1e-3,
                 alpha: float = 0.99, eps: float = 1e-8):
    """RMSProp (the optimizer the paper uses for the shape network, appendix A1.2)."""
    v = alpha * v + (1.0 - alpha) * g * g
    w = w - lr * g / (np.sqrt(v) + eps)
    return w, v


# ------------------------------------------------------------------ CBN + SoftZ lifting
# The occupancy network of the paper's final model (appendix, "Depth Representation" and
# "Pixel-aligned 3D Lifting"; Tab. 2 rows HRNet-CBN and HRNet-CBN-SoftZ).  Reading (the
# figure that draws the network is not in the text): n_blocks blocks of [linear layer,
# conditional batch norm conditioned on the pixel-aligned feature c, ReLU], the first
# linear layer reading the soft one-hot depth code; then a linear head.  Batch norm uses
# the running statistics (inference).  With 5 blocks of width 128, n_z = 64 and 256
# feature channels this is 803,072 FLOP per point (3.29 GFLOP per 4096 calls; Tab. 2 gives
# 3.0).

def softz(z: np.ndarray, n_z: int = 64) -> np.ndarray:
    """Soft one-hot depth code (appendix, the SoftZ equation): with s = (N-1) P'_z and
    P'_z = (P_z + 1) / 2, Z_floor(s) = 1 + floor(s) - s, Z_floor(s)+1 = s - floor(s),
    all other entries 0.  The code is defined for -1 <= P_z <= 1; depths outside are
    clamped to that interval (reading)."""
    z = np.clip(np.asarray(z, np.float64), -1.0, 1.0)
    s = (n_z - 1) * 0.5 * (z + 1.0)
    j = np.floor(s).astype(np.int64)
    frac = s - j
    out = np.zeros((z.size, n_z))
    rows = np.arange(z.size)
    out[rows, np.clip(j, 0, n_z - 1)] = 1.0 + j - s
    hi = j + 1 < n_z
    out[rows[hi], j[hi] + 1] = frac[hi]
    return out


def cbn_logit(net, f: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Logit of the CBN lifting network for features f (n x C) and depths z (n):
    f_out = gamma(c) (f_in - mu) / sqrt(sigma^2 + eps) + beta(c) per block, c = f."""
    f = np.asarray(f, np.float64)
    h = softz(z, net.n_z) @ np.asarray(net.Wp, np.float64).T + net.bp
    for i in range(net.n_blocks):
        if i > 0:
            h = a @ np.asarray(net.W[i - 1], np.float64).T + net.b[i - 1]
        gamma = f @ np.asarray(net.Wg[i], np.float64).T + net.bg[i]
        beta = f @ np.asarray(net.Wb[i], np.float64).T + net.bb[i]
        hn = (h - np.asarray(net.mean[i], np.float64)) / np.sqrt(
            np.asarray(net.var[i], np.float64) + net.eps)
        a = np.maximum(gamma * hn + beta, 0.0)
    return (a @ np.asarray(net.Wo, np.float64).T + net.bo)[:, 0]


def cbn_flops_per_point(net) -> int:
    w, c = net.width, net.feat_dim
    return (2 * net.n_z * w + 2 * w * w * (net.n_blocks - 1) + net.n_blocks * 2 * (2 * c * w)
            + 2 * w)


# ------------------------------------------------------------------ mesh hand-off
# Marching Cubes over the surface cells (the PIFu baseline's mesh extraction, Sec. 1 and
# Sec. 3.2 "Inference for Human Reconstruction"), with the triangulation of each of the
# 256 corner cases derived here from the contour on the cube's faces.
#
# Conventions (readings; the paper only names the algorithm):
#   * corner c of a cell has offsets (dx, dy, dz) = (c >> 2 & 1, c >> 1 & 1, c & 1);
#     local edge e = 4 * axis + 2 * u + v, where (u, v) are the cell offsets of the edge's
#     lower corner along the two other axes in increasing axis order;
#   * a face whose four corners alternate inside/outside (ambiguous) keeps its inside
#     corners apart: each inside corner is cut off by its own segment.  The choice depends
#     on the face alone, so two cells sharing a face cut it alike and the mesh is closed;
#   * each face segment is directed so that, seen from outside the cube, the inside
#     corners lie on its left; the segments of a case join into closed loops, each listed
#     from its smallest local edge; a loop is cut into the fan (v0, v_i+1, v_i) from the
#     first position v0 (in loop order) whose fan has no triangle lying in one face of the
#     cube, so every triangle's normal (right-hand rule) points from inside (label 1) to
#     outside;
#   * loops are emitted by increasing smallest edge; cells in the order of the cell list;
#   * one vertex per lattice edge whose end labels differ, at the 0.5 crossing of the
#     linear interpolation of the two end occupancies (t clipped to [0, 1], t = 1/2 when
#     they are equal); vertices are ordered by global edge id 3 * node + axis.


def _mc_edge_corners(e: int) -> Tuple[int, int]:
    axis, u, v = e // 4, (e >> 1) & 1, e & 1
    others = [a for a in range(3) if a != axis]
    lo = [0, 0, 0]
    lo[others[0]], lo[others[1]] = u, v
    hi = list(lo)
    hi[axis] = 1
    enc = lambda q: 4 * q[0] + 2 * q[1] + q[2]
    return enc(lo), enc(hi)


def _mc_corner_pos(c: int) -> np.ndarray:
    return np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1], np.float64)


def mc_case_triangles(case: int) -> List[Tuple[int, int, int]]:
    """Triangles (local edge triples) of one corner case (bit c set: corner c inside)."""
    inside = [(case >> c) & 1 for c in range(8)]
    edges = [_mc_edge_corners(e) for e in range(12)]
    mid = [(_mc_corner_pos(a) + _mc_corner_pos(b)) / 2 for a, b in edges]
    nxt = {}
    for axis in range(3):
        for side in (0, 1):
            normal = np.zeros(3)
            normal[axis] = 1.0 if side else -1.0
            corners = [c for c in range(8) if ((c >> (2 - axis)) & 1) == side]
            fedges = [e for e in range(12) if e // 4 != axis and
                      all(((c >> (2 - axis)) & 1) == side for c in edges[e])]
            cross = [e for e in fedges if inside[edges[e][0]] != inside[edges[e][1]]]
            ins = [c for c in corners if inside[c]]
            if not cross:
                continue
            if len(cross) == 2:
                segs = [(cross[0], cross[1], ins[0])]
            else:   # ambiguous face: cut off each inside corner
                segs = []
                for c in ins:
                    a, b = [e for e in cross if c in edges[e]]
                    segs.append((a, b, c))
            for a, b, q in segs:
                d = mid[b] - mid[a]
                if np.dot(np.cross(normal, d), _mc_corner_pos(q) - mid[a]) < 0:
                    a, b = b, a
                assert a not in nxt
                nxt[a] = b
    tris = []
    seen = set()
    for start in sorted(nxt):
        if start in seen:
            continue
        loop = [start]
        seen.add(start)
        e = nxt[start]
        while e != start:
            loop.append(e)
            seen.add(e)
            e = nxt[e]
        # fan origin: the first loop position (from the smallest edge, in loop order)
        # whose fan has no triangle lying in one face of the cube (such a triangle would
        # overlap the neighbouring cell's cut of that face); every case has one
        def fan(st):
            L = loop[st:] + loop[:st]
            return [(L[0], L[i + 1], L[i]) for i in range(1, len(L) - 1)]
        for st in range(len(loop)):
            cand = fan(st)
            if not any(_mc_common_face(t) for t in cand):
                tris.extend(cand)
                break
        else:
            raise AssertionError("no fan origin for case %d" % case)
    return tris


def _mc_common_face(tri) -> bool:
    """The three edges of a triangle lie in one face of the cube."""
    common = None
    for e in tri:
        a, b = _mc_edge_corners(e)
        fs = {(ax, sd) for ax in range(3) for sd in (0, 1)
              if ((a >> (2 - ax)) & 1) == sd and ((b >> (2 - ax)) & 1) == sd}
        common = fs if common is None else common & fs
    return bool(common)


def mc_table() -> List[List[Tuple[int, int, int]]]:
    return [mc_case_triangles(c) for c in range(256)]


def mesh_from_grid(occ: np.ndarray, labels: np.ndarray) -> Dict[str, np.ndarray]:
    """Vertices (NDC, float64), their global edge ids and the triangles (vertex index
    triples) of the labelled grid, cell by cell in sorted cell order."""
    n = labels.shape[0]
    R = n - 1
    lab = labels.astype(bool)
    occ = np.asarray(occ, np.float64)
    ids, pos = [], []
    for axis in range(3):
        lo = [slice(0, n)] * 3
        hi = [slice(0, n)] * 3
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        crossed = lab[tuple(lo)] != lab[tuple(hi)]
        for i, j, k in np.argwhere(crossed):
            a = np.array([i, j, k])
            b = a.copy()
            b[axis] += 1
            pa, pb = occ[tuple(a)], occ[tuple(b)]
            t = 0.5 if pb == pa else min(max((0.5 - pa) / (pb - pa), 0.0), 1.0)
            Pa = -1.0 + 2.0 * a / R
            Pb = -1.0 + 2.0 * b / R
            ids.append(((i * n + j) * n + k) * 3 + axis)
            pos.append(Pa + t * (Pb - Pa))
    order = np.argsort(np.array(ids, np.int64), kind="stable")
    ids = np.array(ids, np.int64)[order]
    verts = np.array(pos, np.float64).reshape(-1, 3)[order]
    table = mc_table()
    tris = []
    for cell in surface_cells(labels):
        i, j, k = int(cell // (R * R)), int((cell // R) % R), int(cell % R)
        case = 0
        for c in range(8):
            if lab[i + ((c >> 2) & 1), j + ((c >> 1) & 1), k + (c & 1)]:
                case |= 1 << c
        for tri in table[case]:
            vs = []
            for e in tri:
                axis, u, v = e // 4, (e >> 1) & 1, e & 1
                off = [0, 0, 0]
                others = [a for a in range(3) if a != axis]
                off[others[0]], off[others[1]] = u, v
                gid = (((i + off[0]) * n + (j + off[1])) * n + (k + off[2])) * 3 + axis
                vs.append(int(np.searchsorted(ids, gid)))
            tris.append(vs)
    return dict(edge_ids=ids, verts=verts, tris=np.array(tris, np.int64).reshape(-1, 3))


def front_depth_index(labels: np.ndarray) -> np.ndarray:
    """Per input-view column (i, j): the largest k with label 1 (the occupied node nearest
    the camera at z = +1), -1 where the column is empty."""
    n = labels.shape[2]
    ks = np.where(labels.astype(bool), np.arange(n)[None, None, :], -1)
    return ks.max(axis=2)


def mesh_vertex_visible(edge_ids: np.ndarray, labels: np.ndarray) -> np.ndarray:
    """A vertex on the edge from node (i, j, k) along an axis is visible from the input
    camera (orthographic, at z = +1) when no occupied node lies in front of it in the
    columns of the edge's two nodes: every column's front node index is <= k."""
    n = labels.shape[0]
    kf = front_depth_index(labels)
    out = np.zeros(edge_ids.size, bool)
    for m, g in enumerate(edge_ids):
        axis = int(g % 3)
        node = int(g // 3)
        i, j, k = node // (n * n), (node // n) % n, node % n
        cols = [(i, j)]
        if axis == 0:
            cols.append((i + 1, j))
        elif axis == 1:
            cols.append((i, j + 1))
        out[m] = all(kf[c] <= k for c in cols)
    return out


def mesh_colors(verts: np.ndarray, visible: np.ndarray, image: np.ndarray,
                color_fld: Field) -> np.ndarray:
    """Vertex colours: the input pixel (bilinear, HWC image in [-1, 1]) for visible
    vertices (the texture paragraph of Sec. 3.1); Eq. 2's colour network at
    [Phi(g_T, P_xy); P_z; 0.5] for the others (the vertex lies on the 0.5 level set)."""
    out = np.empty((verts.shape[0], 3))
    if np.any(visible):
        out[visible] = bilinear_sample(image, verts[visible, 0], verts[visible, 1])
    hid = ~visible
    if np.any(hid):
        P = verts[hid]
        f = bilinear_sample(color_fld.feat, P[:, 0], P[:, 1])
        extras = np.stack([P[:, 2], np.full(P.shape[0], 0.5)], 1)
        out[hid] = np.tanh(mlp_preact(color_fld.mlp, f, extras))
    return out


# ------------------------------------------------------------------ point-OHEM (Sec. 3.3)
# Readings: the inverse probability is capped at OHEM_W_MAX (the paper only asks that it
# stay finite); weights enter the sampler as fixed-point integers floor(w * 2^16), so the
# prefix sums are exact; draws come from the counter-based SplitMix64 generator.
OHEM_W_MAX = 2.0 ** 20
OHEM_Q_SCALE = 2 ** 16
_M64 = (1 << 64) - 1
_GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def ohem_point_weight(loss: np.ndarray, alpha: float = 0.7, beta: float = 0.0) -> np.ndarray:
    """Eq. 6 (right): inverse sampling probability of a point from its BCE loss,
    P_pt^-1 = 1 / (exp(-L / alpha) + beta), capped at OHEM_W_MAX."""
    with np.errstate(divide="ignore"):
        w = 1.0 / (np.exp(-np.asarray(loss, np.float64) / alpha) + beta)
    return np.minimum(w, OHEM_W_MAX)


def splitmix64(seed: int, counter: int) -> int:
    """Output number `counter` (0-based) of SplitMix64 (Steele, Lea and Flood 2014)
    started from state `seed`: the state advanced counter + 1 times by the golden gamma,
    then the published finaliser (xor-shift 30, multiply, xor-shift 27, multiply,
    xor-shift 31)."""
    z = (seed + (counter + 1) * _GOLDEN_GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def ohem_sample(weights: np.ndarray, batch: int, seed: int, counter: int) -> np.ndarray:
    """Indices of one training batch drawn with replacement with probability proportional
    to the stored inverse probabilities (their normalisation, Sec. 3.3).  Weights are
    taken as float32 and quantised to q_m = floor(w_m 2^16); draw b uses
    r_b = splitmix64(seed, counter * batch + b), the target t_b = floor(r_b S / 2^64)
    with S = sum q, and picks the first m whose inclusive prefix sum exceeds t_b."""
    w32 = np.asarray(weights, np.float32).astype(np.float64)
    q = np.floor(w32 * OHEM_Q_SCALE).astype(np.uint64)
    S = np.cumsum(q, dtype=np.uint64)
    total = int(S[-1])
    out = np.empty(batch, np.int64)
    for b in range(batch):
        r = splitmix64(seed, counter * batch + b)
        t = (r * total) >> 64
        out[b] = int(np.searchsorted(S, np.uint64(t), side="right"))
    return out


# ------------------------------------------------------------------ number formats

def to_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even); returns float32."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    nan = np.isnan(np.asarray(x, np.float32))
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    out = np.where(nan, np.float32(np.nan), out)
    return out


E4M3_MAX = 448.0


def to_e4m3(x: np.ndarray) -> np.ndarray:
    """Round to OCP FP8 E4M3FN (4 exponent bits, bias 7, 3 mantissa bits, no inf),
    nearest-even, saturating at +-448.  Returns the decoded values as float64."""
    x = np.asarray(x, np.float64)
    a = np.abs(x)
    out = np.zeros_like(a)
    nz = a > 0
    # exponent of the value, clamped to the smallest normal exponent (-6) so that
    # subnormals share the 2^-9 quantum
    e = np.floor(np.log2(np.where(nz, a, 1.0)))
    e = np.maximum(e, -6.0)
    q = np.ldexp(1.0, (e - 3).astype(np.int64))     # spacing of representable values
    m = a / q
    r = np.floor(m)
    frac = m - r
    up = (frac > 0.5) | ((frac == 0.5) & (np.mod(r, 2) == 1))
    r = r + up
    out = np.where(nz, r * q, 0.0)
    out = np.minimum(out, E4M3_MAX)
    out = np.where(np.isnan(x), np.nan, np.sign(x) * out)
    return out
