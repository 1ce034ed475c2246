"""fpo_render_noalloc (the skip modes' scratch in the library's static device
array) against fpo_render with a caller workspace: two calls in a row, the
second with a smaller input, in both skip modes.  The kernels are the same,
so images and transmittances must be equal bit for bit."""
import math

import numpy as np
import pytest

from paper_2202_08614_amd import _lib, synth
from tests.gpu_util import note, require_gpu

pytestmark = pytest.mark.gpu


def test_render_noalloc_matches_render_with_workspace():
    import torch
    dev = require_gpu()
    dijk = synth.blob_leaves(7, 40000)
    k = synth.gaussian_coeffs(len(dijk), seed=77)
    tree = _lib.DeviceTree.from_leaves(dijk, k, 7, device=dev)
    bits = torch.from_numpy(_lib.coarse_occupancy(dijk, 7).view(np.int32)).to(dev)
    packed = _lib.mlp_pack(torch.from_numpy(synth.mlp_init(31)).to(dev))
    calls = [
        # 3 cameras of 1080p: the static array holds 2 per launch, so this is 2 launches
        [synth.ring_camera(0.3 + 1.7 * j, math.radians(5 + 6 * j), 1.5, 30.0, 1920, 1080, 4.0 + 9.0 * j)
         for j in range(3)],
        # then a smaller input: 2 cameras of 320x200 in one launch
        [synth.ring_camera(2.0 + 0.9 * j, math.radians(12 - 8 * j), 1.5, 30.0, 320, 200, 31.0 + 5.0 * j)
         for j in range(2)],
    ]
    for flags in (_lib.FPO_RENDER_SKIP_COARSE, _lib.FPO_RENDER_SKIP_PROPOSAL):
        for cams in calls:
            W, H = cams[0].width, cams[0].height
            ws = _lib.skip_workspace(len(cams), H, W, dev)
            opts = _lib.make_opts(stop_T=1e-3, flags=flags, coarse_bits=bits, proposal=packed, workspace=ws)
            note(f"fpo_render_noalloc flags={flags} {len(cams)} x {W}x{H}")
            want, want_T = _lib.render(tree, cams, opts, want_T=True)
            got, got_T = _lib.render_noalloc(tree, cams, _lib.make_opts(stop_T=1e-3, flags=flags, coarse_bits=bits,
                                                                        proposal=packed), want_T=True)
            torch.cuda.synchronize()
            assert float(want.max()) > 0.05
            assert torch.equal(got, want), float((got - want).abs().max())
            assert torch.equal(got_T, want_T)
