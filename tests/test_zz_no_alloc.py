"""gs_loss_noalloc (the loss with its partial sums in a fixed device array) against gs_loss
(the same kernels on a map's workspace), through the C ABI: identical loss and gradient on
two calls in a row, the second with a smaller image, and an oversized image refused."""
import numpy as np
import pytest

from gpu_common import gpu_map, torch_mod
from paper_2404_06926_amd import gslic, scenes

pytestmark = pytest.mark.gpu


def _pair(H, W, seed):
    rng = np.random.default_rng(seed)
    gt = scenes.smooth_image(seed, H, W)
    out = np.clip(gt + rng.normal(0, 0.05, gt.shape), 0, 1).astype(np.float32)
    torch = torch_mod()
    return torch.tensor(out, device="cuda"), torch.tensor(gt, device="cuda")


def test_loss_noalloc_matches_gs_loss_on_consecutive_calls():
    torch = torch_mod()
    m = gpu_map(np.zeros((0, 14), np.float32), 0)
    # the larger image first, then a smaller ragged one: the second call must not see the
    # first call's partial sums
    for (H, W), seed in [((720, 1280), 21), ((75, 100), 22)]:
        out, gt = _pair(H, W, seed)
        lo_ref, g_ref = m.loss(out, gt, 0.2)
        lo = torch.full((1,), float("nan"), device="cuda")
        g = torch.full_like(out, float("nan"))
        gslic.loss_noalloc(out, gt, 0.2, lo, g)
        torch.cuda.synchronize()
        print(f"{H}x{W}: loss {lo.item():.7f} vs {lo_ref.item():.7f}", flush=True)
        assert torch.equal(lo, lo_ref)
        assert torch.equal(g, g_ref)


def test_loss_noalloc_refuses_images_beyond_its_scratch():
    torch = torch_mod()
    out = torch.zeros(3, 1, 1, device="cuda")
    lo = torch.zeros(1, device="cuda")
    L = gslic.lib()
    # 8192 x 4096 needs 32768 tiles of 32x32: twice the fixed array
    code = L.gs_loss_noalloc(gslic._ptr(out), gslic._ptr(out), 4096, 8192, 0.2, gslic._ptr(lo), gslic._ptr(out),
                             gslic._stream())
    assert code == gslic.GS_ERR_CAPACITY
    assert b"too large" in L.gs_last_error()
