"""Direct fine-tuning of a Fourier PlenOctree on posed images (Sec. 4.3).

One step: draw a batch of (image, row, column) samples, generate their rays
(fpo_camera_rays), render them (fpo_render_rays), take the L2 photometric
loss of Eq. 13 against the images (fpo_l2_loss), back-propagate into the
leaf coefficients (fpo_render_backward) and apply Adam (fpo_adam_step).
Each image carries its own camera and time.  With record=True the forward
keeps each ray's segments (FPO_RAYS_RECORD, up to record_cap per ray) and the
backward works through them segment by segment instead of walking the rays
again.  With graph=True the step (rays, render, loss, backward, Adam with its
step count on the device) is captured once in a HIP graph and replayed.
adam="touched" replaces the dense Adam step by the lazy one
(fpo_adam_step_touched): records the batch's rays did not reach keep their
values and moments.  save() / load() checkpoint and resume a run.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np
import torch

from . import _lib


class FineTuner:
    def __init__(self, tree: _lib.DeviceTree, images: torch.Tensor, cams: Sequence, stop_T: float = 1e-3,
                 lr: float = 1e-2, batch: int = 8192, seed: int = 2022, record: bool = True,
                 record_cap: int = 128, graph: bool = False, adam: str = "dense", two_level: bool = True):
        dev = tree.children.device
        if adam not in ("dense", "touched"):
            raise ValueError("adam must be 'dense' or 'touched'")
        self.adam = adam
        # two_level: the walks descend two levels per read through the tree's
        # two-level table (built here once: the structure never changes while
        # the coefficients are trained); the segments are the same
        if two_level and tree.grandchildren is None and tree.upper() > 0:
            tree = _lib.tree_with_children(tree, tree.children, _lib.grandchild_tables(tree)[0])
        self.tree = tree
        self.images = images
        self.n_img, self.H, self.W = int(images.shape[0]), int(images.shape[1]), int(images.shape[2])
        self.cam_table = torch.from_numpy(_lib.camera_pack(cams)).to(dev)
        times = sorted({float(c.time) for c in cams})
        self.basis = torch.from_numpy(_lib.time_basis(times, tree.layout)).to(dev)
        self.img_t = torch.tensor([times.index(float(c.time)) for c in cams], dtype=torch.int32, device=dev)
        self.batch = int(batch)
        self.record = bool(record) and self.batch <= 32768
        if self.record:
            self.workspace = _lib.record_workspace(self.batch, record_cap, dev)
            self.opts = _lib.make_opts(stop_T=stop_T, flags=_lib.FPO_RAYS_RECORD, workspace=self.workspace)
        else:
            self.workspace = None
            self.opts = _lib.make_opts(stop_T=stop_T)
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)
        self.grad = torch.zeros_like(tree.coeffs)
        self.m = torch.zeros_like(tree.coeffs)
        self.v = torch.zeros_like(tree.coeffs)
        self.lr = float(lr)
        self.t = 0
        n = self.batch
        self.o = torch.empty((n, 3), dtype=torch.float32, device=dev)
        self.d = torch.empty((n, 3), dtype=torch.float32, device=dev)
        self.rgb = torch.empty((n, 3), dtype=torch.float32, device=dev)
        self.grad_rgb = torch.empty((n, 3), dtype=torch.float32, device=dev)
        # graph=True: the whole step with Adam is captured once in a HIP graph and replayed;
        # a batch is copied into static buffers first, and Adam's step count lives on the device
        self.graph = bool(graph)
        self._graph = None
        if self.graph:
            self.adam_state = torch.zeros(4, dtype=torch.int32, device=dev)
            self.g_in = [torch.zeros(n, dtype=torch.int32, device=dev) for _ in range(4)]   # img, py, px, t_idx
            self.g_loss = torch.zeros(1, dtype=torch.float32, device=dev)

    @classmethod
    def from_scene(cls, leaf_dijk: np.ndarray, gt_coeffs: np.ndarray, init_coeffs: np.ndarray, max_depth: int,
                   cams: Sequence, dev, sigma_scale: float = 64.0, stop_T: float = 1e-3, lr: float = 1e-2,
                   batch: int = 8192, seed: int = 2022, record: bool = True, record_cap: int = 128,
                   graph: bool = False, adam: str = "dense", two_level: bool = True) -> "FineTuner":
        """Targets are rendered from the ground-truth coefficients by fpo_render."""
        gt = _lib.DeviceTree.from_leaves(leaf_dijk, gt_coeffs, max_depth, device=dev, sigma_scale=sigma_scale)
        images, _ = _lib.render(gt, cams, _lib.make_opts(stop_T=stop_T))
        del gt
        tree = _lib.DeviceTree.from_leaves(leaf_dijk, init_coeffs, max_depth, device=dev, sigma_scale=sigma_scale)
        return cls(tree, images, cams, stop_T=stop_T, lr=lr, batch=batch, seed=seed, record=record,
                   record_cap=record_cap, graph=graph, adam=adam, two_level=two_level)

    def sample(self):
        """A batch: image, row and column of each ray, and the time index of its image."""
        dev = self.images.device
        n = self.batch
        img = torch.randint(0, self.n_img, (n,), generator=self.gen, device=dev, dtype=torch.int32)
        py = torch.randint(0, self.H, (n,), generator=self.gen, device=dev, dtype=torch.int32)
        px = torch.randint(0, self.W, (n,), generator=self.gen, device=dev, dtype=torch.int32)
        return img, py, px, self.img_t[img.long()]

    def _forward_backward(self, img, py, px, t_idx, loss_out):
        _lib.camera_rays(self.cam_table, img, py, px, self.o, self.d)
        _lib.render_rays(self.tree, self.o, self.d, t_idx, self.basis, self.opts, rgb=self.rgb)
        _lib.l2_loss(self.rgb, self.images, img, py, px, grad_rgb=self.grad_rgb, loss=loss_out)
        _lib.render_backward(self.tree, self.o, self.d, t_idx, self.basis, self.rgb, self.grad_rgb, self.grad,
                             self.opts)

    def step(self, img, py, px, loss_out: torch.Tensor, with_adam: bool = True, t_idx=None):
        if t_idx is None:
            t_idx = self.img_t[img.long()]
        if self.graph and with_adam:
            for dst, src in zip(self.g_in, (img, py, px, t_idx)):
                dst.copy_(src)
            self.g_loss.zero_()
            if self._graph is None:
                torch.cuda.synchronize()
                self._graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(self._graph):
                    self._forward_backward(*self.g_in, self.g_loss)
                    if self.adam == "touched":
                        _lib.adam_step_touched(self.tree.coeffs, self.grad, self.m, self.v, lr=self.lr,
                                               state=self.adam_state)
                    else:
                        _lib.adam_step_dev(self.tree.coeffs, self.grad, self.m, self.v, self.adam_state,
                                           lr=self.lr)
            self._graph.replay()
            loss_out.add_(self.g_loss)
            self.t += 1
            return
        self._forward_backward(img, py, px, t_idx, loss_out)
        if with_adam:
            self.t += 1
            if self.adam == "touched":
                _lib.adam_step_touched(self.tree.coeffs, self.grad, self.m, self.v, step=self.t, lr=self.lr)
            else:
                _lib.adam_step(self.tree.coeffs, self.grad, self.m, self.v, self.t, lr=self.lr)

    # -- checkpoint / resume ------------------------------------------------
    def state_dict(self) -> dict:
        """Everything a resumed run needs: the coefficient records, Adam's
        moments and step count (also the device count of the graph variant),
        and the batch sampler's generator state.  Tensors are copies."""
        sd = {"coeffs": self.tree.coeffs.detach().clone(), "m": self.m.clone(), "v": self.v.clone(),
              "t": torch.tensor(self.t, dtype=torch.int64), "gen": self.gen.get_state()}
        if self.graph:
            sd["adam_state"] = self.adam_state.clone()
        return sd

    def load_state_dict(self, sd: dict) -> None:
        if tuple(sd["coeffs"].shape) != tuple(self.tree.coeffs.shape):
            raise ValueError("checkpoint is for another tree")
        with torch.no_grad():
            self.tree.coeffs.copy_(sd["coeffs"])
            self.m.copy_(sd["m"])
            self.v.copy_(sd["v"])
            self.grad.zero_()
        self.t = int(sd["t"])
        self.gen.set_state(sd["gen"].cpu())
        if self.graph:
            if "adam_state" in sd:
                self.adam_state.copy_(sd["adam_state"])
            else:   # resume an eager run in graph mode: the device count is the step count
                self.adam_state.zero_()
                self.adam_state[0] = self.t
                b1, b2 = 0.9, 0.999
                c = torch.tensor([1.0 / (1.0 - b1 ** max(self.t, 1)), 1.0 / (1.0 - b2 ** max(self.t, 1))],
                                 dtype=torch.float32)
                self.adam_state[1:3] = c.view(torch.int32).to(self.adam_state.device)

    def save(self, path: str) -> None:
        torch.save(self.state_dict(), path)

    def load(self, path: str) -> None:
        """Resume from save(); the file holds tensors only (loaded with weights_only=True)."""
        self.load_state_dict(torch.load(path, map_location="cpu", weights_only=True))

    def train(self, n_steps: int) -> List[float]:
        losses = torch.zeros(n_steps, dtype=torch.float32, device=self.images.device)
        for s in range(n_steps):
            img, py, px, t_idx = self.sample()
            self.step(img, py, px, losses[s:s + 1], t_idx=t_idx)
        return losses.cpu().tolist()
