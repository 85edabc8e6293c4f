"""The allocation-free forward (jtfs_forward_noalloc, for callers that cannot
allocate) against jtfs_forward with a caller workspace, through the C ABI: two
calls in a row on the library's fixed scratch, the second with fewer signals,
and a batch whose workspace exceeds the scratch (rejected before any launch)."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_2204_08269_amd import _lib
from paper_2204_08269_amd.jtfs import JTFS

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _forward_both(op, x):
    """(S1, S2) of jtfs_forward with a torch workspace and of jtfs_forward_noalloc."""
    L = op.lib
    B = x.shape[0]
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    outs = []
    for noalloc in (False, True):
        s1 = torch.full((B,) + op.s1_shape, float("nan"), device=x.device)
        s2 = torch.full((B,) + op.s2_shape, float("nan"), device=x.device)
        if noalloc:
            rc = L.jtfs_forward_noalloc(op.plan, _p(x), B, _p(s1), _p(s2), st)
        else:
            ws = op.new_workspace(B)
            rc = L.jtfs_forward(op.plan, _p(x), B, _p(s1), _p(s2), _p(ws), ws.numel(), st)
        _lib.check(rc)
        torch.cuda.synchronize()
        outs.append((s1.cpu().numpy(), s2.cpu().numpy()))
    return outs


@pytest.mark.parametrize("cfg,contraction,batches", [(1, None, (8, 3)), (2, "split16", (1, 1)),
                                                     (2, "fp32", (1, 1))])
def test_noalloc_forward_matches_workspace_forward(cfg, contraction, batches):
    p = synth.PARAMS[cfg]
    op = JTFS(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"], contraction=contraction)
    assert op.forward_workspace_bytes(max(batches)) <= _lib.JTFS_NOALLOC_SCRATCH_BYTES
    x = torch.from_numpy(synth.batch(cfg, B=max(batches) + 1)).cuda()
    # two calls in a row; the second smaller (or other signals) over the first's scratch contents
    for k, B in enumerate(batches):
        xb = x[k:k + B].contiguous()
        (a1, a2), (b1, b2) = _forward_both(op, xb)
        assert np.isfinite(b1).all() and np.isfinite(b2).all()
        np.testing.assert_array_equal(b1, a1)
        np.testing.assert_array_equal(b2, a2)


def test_noalloc_rejects_batches_beyond_the_scratch():
    p = synth.PARAMS[2]
    op = JTFS(p["N"], p["J"], p["Q"], p["J_fr"], p["Q_fr"], p["T"], p["F"])
    B = 64
    assert op.forward_workspace_bytes(B) > _lib.JTFS_NOALLOC_SCRATCH_BYTES
    x = torch.zeros((B, p["N"]), device="cuda")
    s1 = torch.zeros((B,) + op.s1_shape, device="cuda")
    s2 = torch.zeros((B,) + op.s2_shape, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = op.lib.jtfs_forward_noalloc(op.plan, _p(x), B, _p(s1), _p(s2), st)
    assert rc == _lib.JTFS_EWORKSPACE
    assert b"exceeds the fixed scratch" in op.lib.jtfs_last_error()
    torch.cuda.synchronize()
    assert float(s1.abs().max()) == 0.0 and float(s2.abs().max()) == 0.0
