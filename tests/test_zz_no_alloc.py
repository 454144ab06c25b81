"""The allocation-free camera render (gf_render_noalloc, workspace in a
file-scope device array) against gf_render with a caller workspace: bitwise
the same image and primary transmittance on two calls in a row, the second
with a smaller camera; a camera larger than the fixed workspace is rejected
before any launch; a render whose samples the fixed workspace cannot hold
runs them unsplit and still gives gf_render's bits."""
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
    descs = (gf.render_desc(spp=4, multiple=True, hg_g=0.3, stochastic=True, seed=3, bin="mixture"),
             gf.render_desc(spp=8, exact_shadow=True, seed=4))
    for (w, h), desc in (((96, 80), descs[0]), ((40, 24), descs[0]), ((96, 80), descs[1]), ((40, 24), descs[1])):
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


@pytest.mark.parametrize("kind", ["single_closed_form_shadow", "multiple_scattering"])
def test_noalloc_unsplit_samples_match_split(kind):
    """A render whose per-sample storage exceeds the fixed workspace keeps
    each chunk's samples in one work unit; gf_render, with a caller workspace
    sized for the split, spreads them over several units (one sample each)
    and sums the stored samples afterwards.  The two images have the same
    bits."""
    gf = require_gpu()
    params, rho = W.scene("tiny256"), W.rho("tiny256")
    scene = gf.Scene(dev(params), rho=rho)
    spp = 12
    if kind == "single_closed_form_shadow":
        desc = gf.render_desc(spp=spp, exact_shadow=True, seed=5)
    else:
        desc = gf.render_desc(spp=spp, multiple=True, hg_g=0.3, seed=5)
    cam = gf.camera(1, width=640, height=560)
    n = cam.width * cam.height
    need = gf.gf_render_workspace_size(scene, cam, desc)
    assert need >= 2 * spp * n * 4 + n * 32  # the caller workspace holds every sample
    got, gT = _noalloc(gf, scene, cam, desc)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    ref, rT = gf.gf_render(scene, cam, desc, ws)
    torch.cuda.synchronize()
    assert torch.equal(got, ref) and torch.equal(gT, rT)
    assert bool(torch.isfinite(ref).all())
