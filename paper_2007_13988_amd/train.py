"""Distillation of the surrogate occupancy network with libpifu's training kernels.

The teacher is the full occupancy MLP; samples are (point, teacher occupancy) pairs
that the hierarchical pipeline itself produces on training frames (the nodes it
evaluates on the coarse levels) plus uniform points.  Forward, loss gradient,
backward and RMSProp all run in libpifu (pifu_mlp_grad, pifu_rmsprop_step); torch
only holds the buffers and assembles index lists.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import pifu as P


class MLPTrainer:
    """Gradients + RMSProp for the network of a DeviceMLP (weights updated in place)."""

    def __init__(self, net: P.DeviceMLP, max_batch: int, lr: float = 1e-3, alpha: float = 0.99,
                 eps: float = 1e-8):
        self.net = net
        self.lr, self.alpha, self.eps = lr, alpha, eps
        self.max_batch = max_batch
        self.dW = [torch.zeros_like(w) for w in net.W]
        self.db = [torch.zeros_like(b) for b in net.b]
        self.vW = [torch.zeros_like(w) for w in net.W]
        self.vb = [torch.zeros_like(b) for b in net.b]
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        n = len(net.W)
        self._dW = (C.c_void_p * n)(*[t.data_ptr() for t in self.dW])
        self._db = (C.c_void_p * n)(*[t.data_ptr() for t in self.db])
        self._vW = (C.c_void_p * n)(*[t.data_ptr() for t in self.vW])
        self._vb = (C.c_void_p * n)(*[t.data_ptr() for t in self.vb])
        self.ws = None

    def _field(self, feat: torch.Tensor) -> P.DeviceField:
        return P.DeviceField(P.FIELD_MLP, feat=feat, mlp=self.net)

    def grad(self, feat: torch.Tensor, pts4: torch.Tensor, stream=None,
             point_loss: Optional[torch.Tensor] = None) -> torch.Tensor:
        """pts4: device float32 (n, 4) = (x, y, z, teacher p).  Fills self.dW/self.db (and
        point_loss, device float32 (n,), with every point's BCE when given)."""
        lib = P.load_library()
        fld = self._field(feat)
        n = pts4.shape[0]
        assert n <= self.max_batch
        if self.ws is None:
            sz = C.c_size_t()
            P._check(lib.pifu_mlp_train_workspace_size(C.byref(fld.struct), self.max_batch,
                                                       C.byref(sz)), "train_workspace_size")
            self.ws = torch.empty(sz.value, dtype=torch.uint8, device="cuda")
        st = lib.pifu_mlp_grad_ex(P.context(), C.byref(fld.struct), pts4.data_ptr(), n, self._dW,
                                  self._db, self.loss.data_ptr(),
                                  point_loss.data_ptr() if point_loss is not None else None,
                                  self.ws.data_ptr(), self.ws.numel(), P._stream(stream))
        P._check(st, "pifu_mlp_grad_ex")
        return self.loss

    def point_loss(self, feat: torch.Tensor, pts4: torch.Tensor, stream=None) -> torch.Tensor:
        """Every point's soft-target BCE under the current weights (gradients are filled
        as a side effect)."""
        out = torch.empty(pts4.shape[0], dtype=torch.float32, device="cuda")
        self.grad(feat, pts4, stream, point_loss=out)
        return out

    def step(self, stream=None) -> None:
        lib = P.load_library()
        st = lib.pifu_rmsprop_step(P.context(), C.byref(self.net.struct), self._dW, self._db,
                                   self._vW, self._vb, self.lr, self.alpha, self.eps,
                                   P._stream(stream))
        P._check(st, "pifu_rmsprop_step")

    def save(self, path: str, step: int = 0, extra: Optional[dict] = None) -> None:
        """Checkpoint: FP32 master weights, RMSProp state and the step count (.npz)."""
        arrs = {}
        for l, (w, b, vw, vb) in enumerate(zip(self.net.W, self.net.b, self.vW, self.vb)):
            arrs[f"W{l}"] = w.cpu().numpy()
            arrs[f"b{l}"] = b.cpu().numpy()
            arrs[f"vW{l}"] = vw.cpu().numpy()
            arrs[f"vb{l}"] = vb.cpu().numpy()
        arrs["step"] = np.array([step], np.int64)
        arrs["hyper"] = np.array([self.lr, self.alpha, self.eps], np.float64)
        for k, v in (extra or {}).items():
            arrs[k] = np.asarray(v)
        np.savez(path, **arrs)

    def load(self, path: str) -> int:
        """Restores a checkpoint written by save(); returns its step count."""
        z = np.load(path)
        for l in range(len(self.net.W)):
            self.net.W[l].copy_(torch.from_numpy(z[f"W{l}"]))
            self.net.b[l].copy_(torch.from_numpy(z[f"b{l}"]))
            self.vW[l].copy_(torch.from_numpy(z[f"vW{l}"]))
            self.vb[l].copy_(torch.from_numpy(z[f"vb{l}"]))
        self.lr, self.alpha, self.eps = (float(x) for x in z["hyper"])
        return int(z["step"][0])

    def to_spec(self, template):
        """Copies the trained weights into a synth-style MLPSpec (host float32)."""
        import copy
        spec = copy.copy(template)
        spec.W = [w.detach().cpu().numpy().copy() for w in self.net.W]
        spec.b = [b.detach().cpu().numpy().copy() for b in self.net.b]
        return spec


def lattice_samples(eval_level: torch.Tensor, occ: torch.Tensor, levels: Sequence[int],
                    log2_final: int) -> torch.Tensor:
    """(x, y, z, p) of the nodes the pipeline evaluated on the given levels."""
    n = (1 << log2_final) + 1
    mask = torch.zeros_like(eval_level, dtype=torch.bool)
    for l in levels:
        mask |= eval_level == l
    idx = torch.nonzero(mask.reshape(-1)).reshape(-1)
    i = idx // (n * n)
    j = (idx // n) % n
    k = idx % n
    out = torch.empty((idx.numel(), 4), dtype=torch.float32, device=eval_level.device)
    s = 2.0 / (n - 1)
    out[:, 0] = -1.0 + s * i.float()
    out[:, 1] = -1.0 + s * j.float()
    out[:, 2] = -1.0 + s * k.float()
    out[:, 3] = occ.reshape(-1)[idx]
    return out


@dataclass
class DistillData:
    feats: List[torch.Tensor]      # per frame HWC feature map (device)
    samples: List[torch.Tensor]    # per frame (n, 4) samples (device)


def make_distill_data(teacher_spec, feats_np: Sequence[np.ndarray], per_frame: int, seed: int,
                      levels=(5, 6, 7), log2_final: int = 8, log2_coarse: int = 5,
                      uniform_frac: float = 0.2) -> DistillData:
    """Runs the plain pipeline on each training frame and keeps its coarse-level
    evaluated nodes (with the teacher's occupancy) plus uniform points."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    feats, samples = [], []
    for F in feats_np:
        fld = P.DeviceField.mlp_field(F, teacher_spec)
        out = P.occupancy_grid(fld, log2_final, log2_coarse, eval_level=True)
        lat = lattice_samples(out["eval_level"], out["occ"], levels, log2_final)
        n_lat = int(per_frame * (1 - uniform_frac))
        pick = torch.randint(0, lat.shape[0], (n_lat,), generator=g, device="cuda")
        lat = lat[pick]
        n_uni = per_frame - n_lat
        uni = torch.rand((n_uni, 3), generator=g, device="cuda") * 2 - 1
        _, _, p = P.eval_points(fld, uni, guard_logit=0.0, occ=True)
        uni4 = torch.cat([uni, p[:, None]], dim=1)
        samples.append(torch.cat([lat, uni4]).contiguous())
        feats.append(fld.feat)
    return DistillData(feats, samples)


def train_surrogate(net: P.DeviceMLP, data: DistillData, steps: int = 4000, batch: int = 65536,
                    lr: float = 3e-3, lr_final: float = 1e-4, seed: int = 0, log_every: int = 0,
                    ohem: bool = False, ohem_alpha: float = 0.7, ohem_beta: float = 0.0):
    """RMSProp on the soft-target BCE.  Step s draws a batch (with replacement) from
    frame s mod n_frames; the learning rate follows a cosine from lr to lr_final.
    ohem: point-OHEM (Sec. 3.3, Eq. 6 right) -- each frame's points are drawn with
    probability proportional to 1 / (exp(-L / alpha) + beta) of their last loss L (1
    before a point is first drawn), in libpifu's kernels; else uniformly."""
    import math
    from .pifu import OhemSampler
    tr = MLPTrainer(net, batch, lr=lr)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    losses = []
    nf = len(data.samples)
    samplers = [OhemSampler(smp, min(batch, smp.shape[0]), seed=seed * 1000 + f,
                            alpha=ohem_alpha, beta=ohem_beta)
                for f, smp in enumerate(data.samples)] if ohem else None
    pl = torch.empty(batch, dtype=torch.float32, device="cuda") if ohem else None
    for step in range(steps):
        tr.lr = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * step / max(steps, 1)))
        f = step % nf
        smp = data.samples[f]
        if ohem:
            pts = samplers[f].draw()
            loss = tr.grad(data.feats[f], pts, point_loss=pl)
            samplers[f].update(pl)
        else:
            sel = torch.randint(0, smp.shape[0], (min(batch, smp.shape[0]),), generator=g,
                                device="cuda")
            loss = tr.grad(data.feats[f], smp[sel].contiguous())
        tr.step()
        if log_every and (step + 1) % log_every == 0:
            losses.append(float(loss.item()))
    return tr, losses
