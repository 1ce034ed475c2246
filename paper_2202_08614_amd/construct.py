"""Fourier PlenOctree from per-frame PlenOctrees (Sec. 4.2): unify the
per-frame structures, carry every frame's values onto the union leaves
(split leaves copy their frame leaf's value), take the per-leaf DFT of
Eq. 10-12 and drop the leaves whose density stays below 1e-3 (Sec. 3).
Every step is a libfpo call; torch only holds device memory."""
from __future__ import annotations

from typing import List

import numpy as np

from . import _lib


def build_fpo(frame_leaves: List[np.ndarray], frame_values: List, max_depth: int, device,
              literal: bool = False, prune: bool = True, period: float = None):
    """frame_leaves[t]: [n_t][4] leaves of frame t; frame_values[t]: device
    [n_t][32] F32 snapshot records (caller order).  Returns
    (DeviceTree with F32 coefficient records, union leaves [L][4] in caller
    order of that tree, diagnostics)."""
    import torch
    T = len(frame_leaves)
    union = _lib.union_leaves(np.concatenate(frame_leaves), max_depth)
    children, perm = _lib.build_tree(union, max_depth)
    cells_slot = torch.from_numpy(np.ascontiguousarray(union[perm])).to(device)
    n = union.shape[0]
    frames = torch.empty((T, n, 32), dtype=torch.float32, device=device)
    n_bad = torch.zeros(1, dtype=torch.int32, device=device)
    for t in range(T):
        ft = _lib.FrameTree(frame_leaves[t], max_depth, device)
        _lib.frame_values(ft, frame_values[t], cells_slot, frames[t], n_bad)
    coeffs, smax = _lib.dft_frames(frames, n, literal=literal)
    del frames
    info = {"union_leaves": int(n), "n_bad": int(n_bad.item())}
    slot_union = union[perm]                                   # cells in slot order
    if prune:
        keep = _lib.prune_leaves(smax.cpu().numpy()[:n])
        info["kept"] = int(len(keep))
        leaves = slot_union[keep]
        k_slot = coeffs.view(coeffs.shape[0], -1)[torch.from_numpy(keep).to(device), :166]
    else:
        leaves = slot_union
        k_slot = coeffs.view(coeffs.shape[0], -1)[:n, :166]
    tree = _lib.DeviceTree.from_leaves(leaves, k_slot.cpu().numpy(), max_depth, device=device,
                                       period=float(period if period is not None else T))
    return tree, leaves, info
