"""PlenOctree fusion (Sec. 3, fine stage; Eq. 3-5).

A static PlenOctree (leaf records [leaf_stride][32]: sigma, then z_{c,j} at
1 + 9c + j) is fused with observations of a radiance field from many views,
one view after another: fpo_fusion_observe walks every pixel ray with the
current values and accumulates the observations per leaf, fpo_fusion_apply
updates every observed leaf once (Eq. 3-5) and clears the accumulators.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import _lib


class Fusion:
    def __init__(self, tree: _lib.DeviceTree, values: torch.Tensor, field, tau: float = 1e-3,
                 weight: Optional[torch.Tensor] = None, count: Optional[torch.Tensor] = None):
        dev = values.device
        n = tree.leaf_stride
        if tuple(values.shape) != (n, 32) or values.dtype != torch.float32:
            raise ValueError("values must be float32 [leaf_stride][32]")
        self.tree = tree
        self.values = values
        self.field = _lib.field_struct(field)
        self.tau = float(tau)
        self.weight = weight if weight is not None else torch.zeros(n, dtype=torch.float32, device=dev)
        self.count = count if count is not None else torch.zeros(n, dtype=torch.int32, device=dev)
        self.acc = torch.zeros((n, _lib.FUSION_ACC), dtype=torch.float32, device=dev)

    def view(self, cam) -> None:
        """Fuse one view: observe with the current values, then update."""
        _lib.fusion_observe(self.tree, self.values, cam, self.field, self.acc, self.tau)
        _lib.fusion_apply(self.values, self.weight, self.count, self.acc, self.tree.n_leaves)

    def run(self, cams: Sequence) -> None:
        for cam in cams:
            self.view(cam)
