"""The allocation-free camera render (gf_render_noalloc, workspace in a
file-scope device array) against gf_render with a caller workspace: bitwise
the same image and primary transmittance on two calls in a row, the second
with a smaller camera; a camera larger than the fixed workspace is rejected
before any launch."""
import pytest
import torch

from gen import workloads as W
from gpu_util import dev, require_gpu

pytestmark = pytest.mark.gpu


def _noalloc(gf, scene, cam, desc, want_T=True):
    """through the C ABI (ctypes binding gf_render_noalloc)"""
    return gf.gf_render_noalloc(scene, cam, desc, want_T=want_T)


def test_noalloc_render_matches_caller_workspace():
    gf = require_gpu()
    params, rho = W.scene("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    desc = gf.render_desc(spp=4, multiple=True, hg_g=0.3, stochastic=True, seed=3, bin="mixture")
    for w, h in ((96, 80), (40, 24)):
        cam = gf.camera(1, width=w, height=h)
        got, gT = _noalloc(gf, scene, cam, desc)
        ws = torch.empty(gf.gf_render_workspace_size(scene, cam, desc), dtype=torch.uint8, device="cuda")
        ref, rT = gf.gf_render(scene, cam, desc, ws)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (w, h)
        assert torch.equal(gT, rT), (w, h)
        assert bool(torch.isfinite(got).all())


def test_noalloc_render_rejects_oversized_camera():
    gf = require_gpu()
    params, rho = W.scene("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    cam = gf.camera(1, width=1032, height=1024)
    with pytest.raises(gf.GfError) as e:
        _noalloc(gf, scene, cam, gf.render_desc(spp=1), want_T=False)
    assert e.value.status == gf._lib.GF_EINVAL
    assert "exceed" in str(e.value)
