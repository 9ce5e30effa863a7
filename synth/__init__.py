"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This module holds no arithmetic of the method itself: it only draws the inputs
(feature maps, MLP weights, analytic shapes, view matrices) that both sides read.
All randomness comes from numpy's PCG64 bit generator seeded explicitly.

Recipe (the paper's workloads stand in as synthetic arrays of the same shape):
  * feature maps: per-channel white N(0,1), smoothed by a periodic Gaussian
    filter of std ``sigma_px`` pixels, then standardised per channel; HWC fp32.
    Shapes follow the encoder outputs of Sec. 3.1 / appendix A1.2
    (256 ch x 128 x 128 for the shape encoder).
  * MLP weights: W ~ N(0, 2 / fan_in) (fan_in includes skip inputs), zero biases
    except an optional output bias; row-major [out][in].  The PIFu-size occupancy
    network additionally carries a depth-slab field on four units per layer
    (depth_slab_mlp): each pixel's feature sets one depth interval, so the surface
    is closed and compact like a body's, and the logit is sharp near it.
  * feature sequences: frame t of a performance is the seed's field moved by
    t * (1.5, 0.7) pixels, mixed with a fresh smooth field (sequence_frame).
  * ellipsoid unions: centres U[-0.4,0.4]^3, semi-axes U[0.15,0.45], rotations
    from normalised Gaussian quaternions.
  * views: yaw rotation about the y axis, no translation (3x4 row-major).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def feature_map(H: int, W: int, C: int, sigma_px: float, seed: int) -> np.ndarray:
    """Smooth Gaussian random field, HWC float32, each channel zero-mean unit-std."""
    g = rng(seed)
    white = g.standard_normal((C, H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    # transfer function of a periodic Gaussian blur with std sigma_px pixels
    tf = np.exp(-2.0 * (math.pi ** 2) * (sigma_px ** 2) * (fx ** 2 + fy ** 2))
    sm = np.real(np.fft.ifft2(np.fft.fft2(white, axes=(1, 2)) * tf[None], axes=(1, 2)))
    sm -= sm.mean(axis=(1, 2), keepdims=True)
    sm /= sm.std(axis=(1, 2), keepdims=True)
    return np.ascontiguousarray(np.transpose(sm, (1, 2, 0)).astype(np.float32))


@dataclass
class MLPSpec:
    """Fully connected network description shared by both sides.

    Layer 0 reads [f; extras]; layer l >= 1 reads [h_{l-1}; f] when skip[l] is
    set, else h_{l-1}.  The last layer is the head (1 or 3 outputs).
    """
    feat_dim: int
    n_extra: int                 # scalar inputs after f in layer 0: z (1) or z, occ (2)
    widths: List[int]            # output width of each layer
    skip: List[bool]             # skip[l]: layer l also reads f (skip[0] ignored)
    hidden_act: str = "relu"     # relu | lrelu
    out_act: str = "sigmoid"     # sigmoid | tanh
    W: List[np.ndarray] = field(default_factory=list)   # float32 [out][in]
    b: List[np.ndarray] = field(default_factory=list)   # float32 [out]

    def in_width(self, l: int) -> int:
        if l == 0:
            return self.feat_dim + self.n_extra
        return self.widths[l - 1] + (self.feat_dim if self.skip[l] else 0)

    def flops_per_point(self) -> int:
        return sum(2 * self.in_width(l) * self.widths[l] for l in range(len(self.widths)))

    def n_params(self) -> int:
        return sum(self.in_width(l) * self.widths[l] + self.widths[l] for l in range(len(self.widths)))


def he_mlp(feat_dim: int, n_extra: int, widths: List[int], skip: List[bool], seed: int,
           hidden_act: str = "relu", out_act: str = "sigmoid", out_bias: float = 0.0) -> MLPSpec:
    spec = MLPSpec(feat_dim, n_extra, list(widths), list(skip), hidden_act, out_act)
    g = rng(seed)
    for l, n_out in enumerate(widths):
        fan_in = spec.in_width(l)
        Wl = g.standard_normal((n_out, fan_in)) * math.sqrt(2.0 / fan_in)
        bl = np.zeros(n_out)
        if l == len(widths) - 1:
            bl[:] = out_bias
        spec.W.append(np.ascontiguousarray(Wl.astype(np.float32)))
        spec.b.append(np.ascontiguousarray(bl.astype(np.float32)))
    return spec


def ellipsoids(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """n x 12 float32: centre (3) then M = diag(1/a) R^T row-major (9).

    q(P) = |M (P - c)|^2 is < 1 inside the ellipsoid.
    """
    g = rng(seed)
    out = np.zeros((n, 12), np.float64)
    for e in range(n):
        c = g.uniform(-0.4, 0.4, 3)
        a = g.uniform(0.15, 0.45, 3) * scale
        q = g.standard_normal(4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ])
        M = np.diag(1.0 / a) @ R.T
        out[e, :3] = c
        out[e, 3:] = M.reshape(-1)
    return out.astype(np.float32)


def sphere_as_ellipsoid(r: float) -> np.ndarray:
    out = np.zeros((1, 12), np.float32)
    out[0, 3:] = (np.eye(3) / r).reshape(-1)
    return out


def yaw_view(theta_deg: float) -> np.ndarray:
    """3x4 row-major [A | t] mapping target-view NDC to input-view NDC (rotation about y)."""
    th = math.radians(theta_deg)
    c, s = math.cos(th), math.sin(th)
    if abs(c) < 1e-12:
        c = 0.0
    if abs(s) < 1e-12:
        s = 0.0
    A = np.array([[c, 0.0, s, 0.0], [0.0, 1.0, 0.0, 0.0], [-s, 0.0, c, 0.0]])
    return A.reshape(-1).astype(np.float32)


# ---------------------------------------------------------------- workloads
PLANE_TINY = np.array([0.3, -0.5, 0.8, -0.1], np.float32)   # logit = a.P + d
SHARPNESS = 8.0


def tiny_features():
    """64 ch x 32 x 32, 4-px correlation (the tiny plain-method workload)."""
    return feature_map(32, 32, 64, 4.0, 101)


def tiny_mlp():
    """(64 feat + z) -> 128 -> 64 -> 1, ReLU hidden, sigmoid out."""
    return he_mlp(64, 1, [128, 64, 1], [False, False, False], 201)


def pifu_features(seed: int = 102):
    """256 ch x 128 x 128 (the shape encoder's output size), 16-px correlation."""
    return feature_map(128, 128, 256, 16.0, seed)


def sequence_frame(H: int, W: int, C: int, sigma_px: float, seed: int, t: int, eps: float = 0.1,
                   step_px=(1.5, 0.7)) -> np.ndarray:
    """Frame t of a video-like feature sequence built on feature_map(H, W, C, sigma_px, seed).

    Every frame (t = 0 included) is the seed's underlying field moved by t * step_px
    pixels (x, y; periodic, sub-pixel Fourier shift), mixed with a fresh smooth field of
    the same spectrum drawn for that frame: sqrt(1 - eps^2) * moved + eps * fresh, then
    re-standardized per channel.  Consecutive frames of one performance are similar in
    this way, unlike independent seeds; eps sets how much new content each frame has.
    """
    g = rng(seed)
    white = g.standard_normal((C, H, W))
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    tf = np.exp(-2.0 * (math.pi ** 2) * (sigma_px ** 2) * (fx ** 2 + fy ** 2))
    phase = np.exp(-2j * math.pi * (fx * step_px[0] * t + fy * step_px[1] * t))
    moved = np.real(np.fft.ifft2(np.fft.fft2(white, axes=(1, 2)) * (tf * phase)[None], axes=(1, 2)))
    moved -= moved.mean(axis=(1, 2), keepdims=True)
    moved /= moved.std(axis=(1, 2), keepdims=True)
    g2 = np.random.Generator(np.random.PCG64([int(seed), int(t) + (1 << 20)]))
    fresh = np.real(np.fft.ifft2(np.fft.fft2(g2.standard_normal((C, H, W)), axes=(1, 2)) * tf[None],
                                 axes=(1, 2)))
    fresh -= fresh.mean(axis=(1, 2), keepdims=True)
    fresh /= fresh.std(axis=(1, 2), keepdims=True)
    sm = math.sqrt(1.0 - eps * eps) * moved + eps * fresh
    sm -= sm.mean(axis=(1, 2), keepdims=True)
    sm /= sm.std(axis=(1, 2), keepdims=True)
    return np.ascontiguousarray(np.transpose(sm, (1, 2, 0)).astype(np.float32))


def pifu_sequence(seed: int, t: int):
    """Frame t of a 256 ch x 128 x 128 feature sequence on the field of pifu_features(seed)."""
    return sequence_frame(128, 128, 256, 16.0, seed, t)


def depth_slab_mlp(spec: MLPSpec, seed: int, kappa: float = 16.0, mu_scale: float = 0.3,
                   tau0: float = -0.05, tau_scale: float = 0.25, eps: float = 0.1) -> MLPSpec:
    """Turns a He-init ReLU occupancy network into a pixel-aligned depth-slab field.

    Hidden units 0-3 of every hidden layer are set to carry
        u0 = relu(z - mu(f)),  u1 = relu(mu(f) - z),  t+ = relu(tau(f)),  t- = relu(-tau(f))
    with mu(f) = mu_scale * a.f and tau(f) = tau0 + tau_scale * b.f (a, b random unit
    vectors): layer 0 computes them, later layers pass them through unchanged (weight 1
    on the unit itself, 0 elsewhere; relu is the identity on them).  The head reads
        logit = kappa * (t+ - t- - u0 - u1 + eps * r),
    i.e. kappa * (tau(f) - |z - mu(f)|) plus eps times the He-init head over the other
    units (r).  Each pixel thus holds one depth interval |z - mu| < tau whose centre and
    half-thickness follow its feature, the way a pixel-aligned occupancy network encodes
    a body, and the field is closed and compact; kappa sets the logit slope
    (kappa * 2 / 2^L per voxel of a 2^L grid).  The other units keep their random weights,
    so the arithmetic per point is unchanged.
    """
    assert len(spec.widths) >= 2 and spec.n_extra >= 1 and spec.hidden_act == "relu"
    g = rng(seed)
    C = spec.feat_dim
    a = g.standard_normal(C)
    a /= np.linalg.norm(a)
    b = g.standard_normal(C)
    b /= np.linalg.norm(b)
    W = [w.astype(np.float64) for w in spec.W]
    B = [x.astype(np.float64) for x in spec.b]
    # layer 0 reads [f; z(; extras)]
    W[0][:4, :] = 0.0
    W[0][0, :C], W[0][0, C] = -mu_scale * a, 1.0
    W[0][1, :C], W[0][1, C] = mu_scale * a, -1.0
    W[0][2, :C] = tau_scale * b
    W[0][3, :C] = -tau_scale * b
    B[0][:4] = [0.0, 0.0, tau0, -tau0]
    n = len(spec.widths)
    for l in range(1, n - 1):
        W[l][:4, :] = 0.0
        for k in range(4):
            W[l][k, k] = 1.0
        B[l][:4] = 0.0
    head = W[n - 1]
    head[:, 4:] *= eps
    head[:, :4] = np.array([-1.0, -1.0, 1.0, -1.0])
    head *= kappa
    B[n - 1] = B[n - 1] * kappa * eps
    spec.W = [np.ascontiguousarray(w.astype(np.float32)) for w in W]
    spec.b = [np.ascontiguousarray(x.astype(np.float32)) for x in B]
    return spec


def pifu_mlp(seed: int = 202, out_bias: float = 0.0):
    """(256+z)->1024->512->256->128->1 with the feature concatenated into hidden layers 2-4;
    a depth-slab occupancy field (see depth_slab_mlp) on He-init weights."""
    spec = he_mlp(256, 1, [1024, 512, 256, 128, 1], [False, True, True, True, False], seed,
                  out_bias=out_bias)
    return depth_slab_mlp(spec, seed + 1)


def surrogate_mlp(seed: int = 203):
    """(256+z)->128->64->1, the distilled occupancy network."""
    return he_mlp(256, 1, [128, 64, 1], [False, False, False], seed)


def color_features(seed: int = 802):
    return feature_map(128, 128, 256, 16.0, seed)


def color_mlp(seed: int = 902):
    """(256 + z + occ) -> 512 -> 256 -> 3, LeakyReLU hidden, tanh out."""
    return he_mlp(256, 2, [512, 256, 3], [False, False, False], seed,
                  hidden_act="lrelu", out_act="tanh")


def precision_points(n: int, seed: int = 403) -> np.ndarray:
    """n uniform points in [-1,1]^3 (float64 n x 3)."""
    return rng(seed).uniform(-1.0, 1.0, (n, 3))


def jitter_points(base: np.ndarray, spacing: float, seed: int) -> np.ndarray:
    g = rng(seed)
    return base + g.uniform(-0.5 * spacing, 0.5 * spacing, base.shape)


@dataclass
class CBNSpec:
    """Weights of the conditional-batch-norm lifting network with soft one-hot depth
    (appendix, "Depth Representation" and "Pixel-aligned 3D Lifting"): a first layer from
    the n_z-channel depth code to `width`, n_blocks blocks of [linear layer (the first one
    is the depth layer), conditional batch norm whose scale and shift are linear maps of
    the pixel-aligned feature, ReLU], and a linear head.  Everything float32."""
    feat_dim: int
    n_z: int
    width: int
    n_blocks: int
    Wp: np.ndarray              # [width][n_z]
    bp: np.ndarray
    W: List[np.ndarray]         # blocks 1 .. n_blocks-1: [width][width]
    b: List[np.ndarray]
    Wg: List[np.ndarray]        # per block [width][feat_dim]: scale gamma(c)
    bg: List[np.ndarray]
    Wb: List[np.ndarray]        # per block [width][feat_dim]: shift beta(c)
    bb: List[np.ndarray]
    mean: List[np.ndarray]      # per block running mean [width]
    var: List[np.ndarray]       # per block running variance [width]
    Wo: np.ndarray              # [1][width]
    bo: np.ndarray              # [1]
    eps: float = 1e-5


def cbn_net(feat_dim: int = 256, n_z: int = 64, width: int = 128, n_blocks: int = 5,
            seed: int = 212, out_bias: float = -2.5) -> CBNSpec:
    """He-initialised linear layers; gamma(c) = 1 + a small linear map of c, beta(c) a
    linear map of c; running statistics near (0, 1); a random head whose constant bias
    (a fixed input, -2.5 by default) puts the surface inside the volume."""
    g = rng(seed)
    f32 = np.float32

    def lin(o, i, std):
        return (g.standard_normal((o, i)) * std).astype(f32)

    W = [lin(width, width, np.sqrt(2.0 / width)) for _ in range(n_blocks - 1)]
    return CBNSpec(
        feat_dim, n_z, width, n_blocks,
        Wp=lin(width, n_z, np.sqrt(2.0)), bp=np.zeros(width, f32),
        W=W, b=[np.zeros(width, f32) for _ in W],
        Wg=[lin(width, feat_dim, 0.1 / np.sqrt(feat_dim)) for _ in range(n_blocks)],
        bg=[np.ones(width, f32) for _ in range(n_blocks)],
        Wb=[lin(width, feat_dim, 1.0 / np.sqrt(feat_dim)) for _ in range(n_blocks)],
        bb=[np.zeros(width, f32) for _ in range(n_blocks)],
        mean=[(g.standard_normal(width) * 0.1).astype(f32) for _ in range(n_blocks)],
        var=[g.uniform(0.5, 1.5, width).astype(f32) for _ in range(n_blocks)],
        Wo=lin(1, width, np.sqrt(1.0 / width)), bo=np.full(1, out_bias, f32))


def depth_slab_cbn(spec: CBNSpec, seed: int, kappa: float = 16.0, mu_scale: float = 0.3,
                   tau0: float = -0.05, tau_scale: float = 0.25, eps: float = 0.1) -> CBNSpec:
    """The depth-slab field of depth_slab_mlp built into a CBN network: units 0-3 of every
    block carry u0 = relu(z - mu(c)), u1 = relu(mu(c) - z), t+ = relu(tau(c)),
    t- = relu(-tau(c)) with mu(c) = mu_scale * a.c and tau(c) = tau0 + tau_scale * b.c.
    The depth layer writes z on units 0 and 1 (the soft one-hot code interpolates the bin
    positions linearly, so Wp[:, j] = -1 + 2 j / (n_z - 1) reproduces P_z exactly) and 0 on
    units 2 and 3; block 0's batch norm is the identity on them (mean 0, variance
    1 - eps_bn) and its conditional scale and shift give the four units (gamma = +1 / -1 /
    0 / 0, beta = -mu / +mu / tau / -tau); later blocks pass them through.  The head reads
    kappa * (t+ - t- - u0 - u1 + eps * r) with r the random head over the other units.
    The same seed as depth_slab_mlp gives the same directions a, b, hence the same slab.
    The other units keep their random weights, so the arithmetic per point is unchanged."""
    assert spec.width >= 4
    g = rng(seed)
    C = spec.feat_dim
    a = g.standard_normal(C)
    a /= np.linalg.norm(a)
    b = g.standard_normal(C)
    b /= np.linalg.norm(b)
    f32 = np.float32
    zpos = -1.0 + 2.0 * np.arange(spec.n_z) / (spec.n_z - 1)
    Wp = spec.Wp.astype(np.float64)
    bp = spec.bp.astype(np.float64)
    Wp[:4, :] = 0.0
    Wp[0, :] = zpos
    Wp[1, :] = zpos
    bp[:4] = 0.0
    W = [w.astype(np.float64) for w in spec.W]
    B = [x.astype(np.float64) for x in spec.b]
    for l in range(len(W)):
        W[l][:4, :] = 0.0
        for k in range(4):
            W[l][k, k] = 1.0
        B[l][:4] = 0.0
    Wg = [w.astype(np.float64) for w in spec.Wg]
    bg = [x.astype(np.float64) for x in spec.bg]
    Wb = [w.astype(np.float64) for w in spec.Wb]
    bb = [x.astype(np.float64) for x in spec.bb]
    mean = [m.astype(np.float64) for m in spec.mean]
    var = [v.astype(np.float64) for v in spec.var]
    for i in range(spec.n_blocks):
        Wg[i][:4, :] = 0.0
        Wb[i][:4, :] = 0.0
        mean[i][:4] = 0.0
        var[i][:4] = 1.0 - spec.eps
        if i == 0:
            bg[i][:4] = [1.0, -1.0, 0.0, 0.0]
            Wb[i][0, :] = -mu_scale * a
            Wb[i][1, :] = mu_scale * a
            Wb[i][2, :] = tau_scale * b
            Wb[i][3, :] = -tau_scale * b
            bb[i][:4] = [0.0, 0.0, tau0, -tau0]
        else:
            bg[i][:4] = 1.0
            bb[i][:4] = 0.0
    Wo = spec.Wo.astype(np.float64)
    Wo[:, 4:] *= eps
    Wo[:, :4] = np.array([-1.0, -1.0, 1.0, -1.0])
    Wo *= kappa
    bo = spec.bo.astype(np.float64) * kappa * eps
    c = lambda x: np.ascontiguousarray(x.astype(f32))
    return CBNSpec(spec.feat_dim, spec.n_z, spec.width, spec.n_blocks, Wp=c(Wp), bp=c(bp),
                   W=[c(w) for w in W], b=[c(x) for x in B], Wg=[c(w) for w in Wg],
                   bg=[c(x) for x in bg], Wb=[c(w) for w in Wb], bb=[c(x) for x in bb],
                   mean=[c(m) for m in mean], var=[c(v) for v in var], Wo=c(Wo), bo=c(bo),
                   eps=spec.eps)


def pifu_cbn(seed: int = 212):
    """The appendix's CBN + SoftZ network at the paper's size (SoftZ n_z = 64, five CBN
    blocks of width 128 on 256 feature channels) carrying the benchmark's depth-slab field
    (the slab of pifu_mlp(): same directions).  The other units are batch-normalised, so
    their head term is larger than the He-init MLP's; eps = 0.02 gives a slab of about the
    same occupancy and surface area."""
    return depth_slab_cbn(cbn_net(seed=seed, out_bias=0.0), 203, eps=0.02)
