"""Learned proposal: training data from the plain walk, GPU training with the
library's MLP kernels, and the packed FP16 weights the render's skip pre-pass
reads.  Every step runs in libfpo; torch only holds device memory."""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import _lib, synth


def training_set(tree: "_lib.DeviceTree", n_rays: int, n_cams: int = 4096, stop_T: float = 1e-3,
                 width: int = 1920, height: int = 1080, seed: int = synth.RAY_SEED, chunk: int = 1 << 20):
    """Labelled rays (labels [n][3], inputs [n][7]) from random ring cameras,
    pixels and times, labelled by fpo_ray_labels."""
    import torch
    dev = tree.children.device
    cams = synth.c5_train_cameras(n_cams, width, height, seed)
    table = torch.from_numpy(_lib.camera_pack(cams)).to(dev)
    grid = synth.c5_time_grid()
    basis = torch.from_numpy(_lib.time_basis(grid)).to(dev)
    tau = torch.from_numpy(np.mod(grid / synth.PERIOD, 1.0).astype(np.float32)).to(dev)
    cam, py, px, t_idx = synth.c5_train_samples(n_rays, n_cams, width, height, seed)
    labels = torch.empty((n_rays, 3), dtype=torch.float32, device=dev)
    inputs = torch.empty((n_rays, _lib.MLP_N_IN), dtype=torch.float32, device=dev)
    opts = _lib.make_opts(stop_T=stop_T)
    for a in range(0, n_rays, chunk):
        b = min(a + chunk, n_rays)
        c_d = torch.from_numpy(cam[a:b]).to(dev)
        y_d = torch.from_numpy(py[a:b]).to(dev)
        x_d = torch.from_numpy(px[a:b]).to(dev)
        o, d = _lib.camera_rays(table, c_d, y_d, x_d)
        ti = torch.from_numpy(t_idx[a:b]).to(dev)
        lab, inp = _lib.ray_labels(tree, o, d, ti, basis, tau, opts)
        labels[a:b] = lab
        inputs[a:b] = inp
    return labels, inputs


class Proposal:
    """FP32 master weights with Adam state on the device."""

    def __init__(self, device, seed: int = 11, params: Optional[np.ndarray] = None):
        import torch
        p = synth.mlp_init(seed) if params is None else np.asarray(params, np.float32)
        if p.size == _lib.MLP_N_PARAMS:
            p = np.concatenate([p, np.zeros(1, np.float32)])
        self.params = torch.from_numpy(p.copy()).to(device)
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.step = 0
        self._ws = None
        self._ws_n = 0

    def train(self, inputs, labels, steps: int, batch: int = 16384, lr: float = 2e-3,
              seed: int = 0, log_every: int = 0) -> List[float]:
        """Adam on random batches; returns the mean batch loss of each logging
        interval (one value at the end when log_every is 0)."""
        import torch
        dev = self.params.device
        if self._ws is None or self._ws_n < batch:
            self._ws = _lib.mlp_workspace(batch, dev)
            self._ws_n = batch
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        n = int(inputs.shape[0])
        hist = []
        every = log_every if log_every > 0 else steps
        self.loss.zero_()
        for i in range(steps):
            idx = torch.randint(0, n, (batch,), generator=gen, device=dev, dtype=torch.int32)
            _lib.mlp_loss_grad(self.params, inputs, labels, self.grad, self.loss, self._ws, idx=idx)
            self.step += 1
            _lib.adam_step(self.params, self.grad, self.m, self.v, self.step, lr=lr)
            if (i + 1) % every == 0:
                hist.append(float(self.loss.item()) / every)
                self.loss.zero_()
        return hist

    def packed(self):
        return _lib.mlp_pack(self.params)
