"""Surrogate form of the pipeline: a distilled small occupancy network on the coarse
levels, the full network at the finest level and wherever the surrogate's
occupancy is within delta_s of 0.5.  Training data, training, delta selection and the
accuracy report all run through libpifu (see train.py)."""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np
import torch

from . import pifu as P
from .train import make_distill_data, train_surrogate


def cell_disagreement(cells: torch.Tensor, ref_cells: torch.Tensor) -> float:
    """|symmetric difference of two sorted surface-cell lists| / |reference cells|."""
    a = cells.to(torch.int64)
    b = ref_cells.to(torch.int64)
    if b.numel() == 0:
        return 0.0 if a.numel() == 0 else float("inf")
    in_b = torch.isin(a, b)
    in_a = torch.isin(b, a)
    diff = int((~in_b).sum().item()) + int((~in_a).sum().item())
    return diff / b.numel()


def full_mlp_points(stats: Sequence[Dict[str, int]]) -> int:
    """Points the full network evaluated (every level's mlp_points, surrogate excluded)."""
    return int(sum(s["mlp_points"] for s in stats))


def distill(teacher_spec, student_spec, feats_train: Sequence[np.ndarray], samples_per_frame: int,
            steps: int = 4000, batch: int = 65536, seed: int = 0, lr: float = 3e-3,
            lr_final: float = 1e-4, ohem: bool = False):
    """Trains student_spec (in place on the GPU) against teacher_spec; returns the
    DeviceMLP of the student and the logged losses.  ohem: point-OHEM sampling."""
    data = make_distill_data(teacher_spec, feats_train, samples_per_frame, seed)
    net = P.DeviceMLP(student_spec)
    tr, losses = train_surrogate(net, data, steps=steps, batch=batch, lr=lr, lr_final=lr_final,
                                 seed=seed, log_every=max(1, steps // 50), ohem=ohem)
    del data
    return net, losses


def choose_delta(teacher_spec, net: P.DeviceMLP, feats_val: Sequence[np.ndarray],
                 deltas=(0.02, 0.05, 0.1, 0.15, 0.2, 0.3, 0.45), bar: float = 1e-3,
                 log2_final=8, log2_coarse=5, sur_max_log2=7, precision="bf16", band_delta=0.02):
    """Smallest delta_s whose surface cells disagree with the plain FP32 grid by at
    most `bar` (fraction of cells) on every validation frame."""
    refs = []
    for F in feats_val:
        fld = P.DeviceField.mlp_field(F, teacher_spec)
        refs.append(P.occupancy_grid(fld, log2_final, log2_coarse)["cells"].clone())
    report = []
    for d in deltas:
        worst = 0.0
        for F, ref in zip(feats_val, refs):
            fld = P.DeviceField(P.FIELD_MLP, feat=F, mlp=P.DeviceMLP(teacher_spec), surrogate=net)
            out = P.occupancy_grid(fld, log2_final, log2_coarse, precision=precision,
                                   band_delta=band_delta, surrogate_max_log2=sur_max_log2,
                                   surrogate_delta=d)
            worst = max(worst, cell_disagreement(out["cells"], ref))
        report.append((d, worst))
        if worst <= bar:
            return d, report
    return deltas[-1], report
