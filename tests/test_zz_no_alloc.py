"""The allocation-free MSE entry point (eelbm_cno_mse_noalloc) against the
workspace one (eelbm_cno_mse): the same loss, bit for bit, and the same
gradient, on two calls in a row (the second smaller, so that stale partial
sums of the first would show), plus the size limit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(B, H, W, C, seed):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    pred = torch.randn(B, H, W, C, generator=g, dtype=torch.float32).cuda()
    target = torch.randn(B, H, W, C, generator=g, dtype=torch.float32).cuda()
    return pred, target


def _with_workspace(pred, target, Cu, nb):
    import torch
    from paper_2409_10399_amd.binding import lib
    P = pred.numel() // pred.shape[-1]
    part = torch.zeros(nb, dtype=torch.float64, device="cuda")
    d = torch.empty_like(pred)
    rc = lib().eelbm_cno_mse(ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(target.data_ptr()), P,
                             pred.shape[-1], Cu, ctypes.c_void_p(part.data_ptr()), nb, ctypes.c_void_p(d.data_ptr()),
                             None)
    assert rc == 0
    torch.cuda.synchronize()
    total = 0.0
    for v in part.cpu().numpy().tolist():     # block order
        total += v
    return total, d.cpu().numpy()


def _noalloc(pred, target, Cu, nb):
    import torch
    from paper_2409_10399_amd.binding import lib
    P = pred.numel() // pred.shape[-1]
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    d = torch.empty_like(pred)
    rc = lib().eelbm_cno_mse_noalloc(ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(target.data_ptr()), P,
                                     pred.shape[-1], Cu, nb, ctypes.c_void_p(loss.data_ptr()),
                                     ctypes.c_void_p(d.data_ptr()), None)
    assert rc == 0, lib().eelbm_last_error()
    torch.cuda.synchronize()
    return float(loss.cpu().item()), d.cpu().numpy()


def test_noalloc_mse_matches_workspace_mse():
    for (B, H, W, C, Cu, nb, seed) in ((4, 64, 64, 16, 6, 1024, 1), (1, 16, 32, 16, 9, 37, 2)):
        pred, target = _case(B, H, W, C, seed)
        l0, d0 = _with_workspace(pred, target, Cu, nb)
        l1, d1 = _noalloc(pred, target, Cu, nb)
        print(f"  B={B} H={H} W={W} nb={nb}: loss {l0!r} / {l1!r}", flush=True)
        assert l1 == l0
        assert np.array_equal(d1, d0)
        ref = float(((pred[..., :Cu].double() - target[..., :Cu].double()) ** 2).mean().cpu())
        assert abs(l1 - ref) <= 1e-12 * ref


def test_noalloc_mse_rejects_oversize():
    from paper_2409_10399_amd.binding import lib
    import torch
    pred, target = _case(1, 8, 8, 16, 3)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    rc = lib().eelbm_cno_mse_noalloc(ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(target.data_ptr()), 64, 16, 6,
                                     1025, ctypes.c_void_p(loss.data_ptr()), None, None)
    assert rc == -2
    assert b"EELBM_CNO_MSE_MAX_BLOCKS" in lib().eelbm_last_error()
