"""The allocation-free splat entry point (splat_render_noalloc, workspace in
the library's fixed device array) against splat_render with a caller
workspace, through the C ABI: two calls in a row, the second with a smaller
input, each bit-identical to the workspace form (same kernels, same layout),
and a request beyond the array's size refused before any work."""
import numpy as np
import pytest

import synth
from paper_0811_2055_amd import lib

from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def test_noalloc_matches_splat_render_twice_then_refuses_oversize():
    import torch
    big = synth.small_clustered(1_000_000, 301)
    small = synth.small_clustered(150_000, 302)
    cams = [lib.Camera.ortho(1024, 1024),
            lib.Camera.look_at((0.5, 0.45, -0.7), (0.5, 0.5, 0.5), 640, 480, fov_deg=60.0)]
    outs = []
    for s, cam in ((big, cams[0]), (small, cams[1])):
        d = to_dev(s)
        print(f"[noalloc] {s.n} points {cam.W}x{cam.H}", flush=True)
        want = lib.splat(*d, cam).cpu().numpy()
        got = lib.splat_noalloc(*d, cam).cpu().numpy()
        assert np.array_equal(got.view(np.int32), want.view(np.int32)), s.n
        assert float(want.max()) > 0
        outs.append(got)
    # beyond the array (3 M points at 1024^2 need about 160 MB): refused with
    # LOD_ECAPACITY, nothing enqueued, output untouched
    huge = 3_000_000
    e = torch.zeros(huge, dtype=torch.float32, device="cuda")
    img = torch.full((1024, 1024), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(lib.LodError) as err:
        lib.splat_noalloc(e, e, e, e, cams[0], out=img)
    assert err.value.code == lib.LOD_ECAPACITY
    assert float(img.min()) == 7.0 and float(img.max()) == 7.0
    # and the array still serves a call afterwards
    d = to_dev(small)
    again = lib.splat_noalloc(*d, cams[1]).cpu().numpy()
    assert np.array_equal(again.view(np.int32), outs[1].view(np.int32))
