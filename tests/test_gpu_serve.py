"""GPU checks of the continuous-batching server: every request completes,
each image is bitwise the same rendered in the mix, alone through the server,
by the plain camera renderer (gf_render, caller workspace) and through the
ray-list call (gf_render_rays); admission never holds
more device memory than the budget; requests that can never fit are
rejected."""
import numpy as np
import pytest
import torch

import gen
from gpu_util import dev, host, require_gpu

pytestmark = pytest.mark.gpu


def _trace(n, seed):
    reqs = gen.serving_requests(n, seed, n_scenes=3)
    for r in reqs:
        r["res"] = {128: 32, 256: 48, 512: 64, 1024: 96}[r["res"]]
    return reqs


def test_server_mix_equals_alone_and_plain():
    gf = require_gpu()
    from paper_2602_05081_amd import serve
    scenes = [gf.Scene(dev(gen.blob_scene(n, s)), rho=r) for n, s, r in
              ((2000, 10, 0.004), (8000, 11, 0.0015), (20000, 12, 0.0008))]
    reqs = _trace(24, 3)
    # a few requests at a time: admission binds (pool bytes: rays, then
    # per-sample radiance)
    need = [r["res"] ** 2 * (32 + 4 * r["spp"]) + 512 for r in reqs]
    budget = max(3 * 48 * 48 * (32 + 16) + 1536, max(need))
    arrivals = np.zeros(len(reqs))
    lat, mk, mix, held = serve.run_server(scenes, reqs, arrivals, mem_budget=budget, tile_rays=512, max_tiles=8,
                                          time_limit=120)
    assert held <= budget
    assert len(lat) == len(reqs)
    for k, r in enumerate(reqs):
        alone = serve.run_server(scenes, [r], np.zeros(1), mem_budget=budget, tile_rays=512, max_tiles=8,
                                 time_limit=60)[2][0]
        assert torch.equal(mix[k], alone), k
        cam, desc = serve.request_camera(r), serve.request_desc(r)
        ws = torch.empty(gf.gf_render_workspace_size(scenes[r["scene"]], cam, desc), dtype=torch.uint8,
                         device="cuda")
        plain, _ = gf.gf_render(scenes[r["scene"]], cam, desc, ws)
        assert torch.equal(mix[k], plain.view(-1)), k
        rays = gf.gf_camera_rays(cam)
        listed, _, _, _ = gf.gf_render_rays(scenes[r["scene"]], rays, desc, image_width=cam.width)
        assert torch.equal(mix[k], listed), k
        assert torch.isfinite(mix[k]).all()


def test_server_rejects_oversized_request():
    gf = require_gpu()
    from paper_2602_05081_amd import serve
    scene = gf.Scene(dev(gen.blob_scene(500, 1)), rho=0.01)
    srv = gf._lib.Server(64 * 64 * 32 + 64 * 64 * 4, 256, 4)
    r = dict(scene=0, res=128, lod=0, spp=1, multiple=0, az=0.0, el=0.0, seed=1)
    out = torch.empty(128 * 128, device="cuda")
    with pytest.raises(gf.GfError):
        srv.submit(scene, serve.request_camera(r), serve.request_desc(r), out)
    srv.close()
