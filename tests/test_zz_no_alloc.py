"""The allocation-free entry point (bf_filter_noalloc) against bf_filter_ws:
the same kernels with the library's per-GPU scratch array as workspace, so
every output must be bitwise the same.  Two calls in a row (the second on a
smaller image, which reuses the array the first one left), and the size limit."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_noalloc_matches_filter_ws(gpu):
    import torch
    from paper_1803_00004_amd import bf
    cases = [(300, 520, 3.0, 9, 4, 0.1, 8, "f32"), (120, 90, 4.0, 12, 6, 0.2, 16, "u8")]
    for H, W, ss, r, ns, sr, nr, dt in cases:
        print("[noalloc] %dx%d r %d %s" % (H, W, r, dt), flush=True)
        plan = bf.Plan(ss, sr, r, nr, ns, dtype=dt)
        need = plan.workspace_size(H, W)
        assert 0 < need <= bf.NOALLOC_SCRATCH_BYTES
        host = synth.gen_image_u8(H, W, 5, 0.03, H + W) if dt == "u8" else synth.gen_image(H, W, 5, 0.03, H + W)
        I = torch.from_numpy(host).cuda()
        ref = bf.filter(plan, I, ws=bf.workspace(plan, H, W))
        out = torch.full((H, W), -1.0, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        bf.filter_noalloc(plan, I, out)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)  # nothing of workspace size was allocated
        assert torch.equal(out, ref)


def test_noalloc_refuses_workspace_above_the_limit(gpu):
    import torch
    from paper_1803_00004_amd import bf
    plan = bf.Plan(16.0, 0.05, 48, 32, 8)
    H = W = 2048
    assert plan.workspace_size(H, W) > bf.NOALLOC_SCRATCH_BYTES
    I = torch.zeros((H, W), device="cuda")
    out = torch.full((H, W), -1.0, device="cuda")
    st = bf.lib().bf_filter_noalloc(plan.handle, ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   H, W, None)
    assert st == bf.BF_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((out == -1.0).all())  # nothing was enqueued
