"""Streaming merge (hmfsr_stream_begin / add / end through the C ABI): frames
added one call at a time into a fixed-size state equal the one-call merge."""
import numpy as np
import pytest
import torch

import oracle.merge as om
from parity_util import assert_parity
from paper_1905_03277_amd import synth, torch_ops

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def stream_merge(b, order):
    f, m = b.frames.to(DEV), b.motion.to(DEV)
    sm = torch_ops.StreamingMerge(f[b.desc.ref_frame].contiguous(), b.desc, b.tuning)
    for n in order:
        sm.add(f[n].contiguous(), m[n].contiguous())
    out = sm.result()
    torch.cuda.synchronize()
    return out.cpu().numpy(), sm


@pytest.mark.parametrize("n,h,w,scale,tile,cfa,ref", [
    (5, 96, 128, 1.5, 16, 0, 0), (3, 70, 102, 2.0, 8, 3, 1), (8, 64, 64, 1.0, 32, 1, 0), (1, 48, 64, 1.25, 16, 2, 0)])
def test_stream_equals_one_call_merge_bitwise(n, h, w, scale, tile, cfa, ref, monkeypatch):
    monkeypatch.setenv("HMFSR_MERGE_VARIANT", "2")     # the 64 x 16 shape the stream uses
    b = synth.make_burst(n, h, w, seed=3100 + n, scale=scale, tile_size=tile, cfa=cfa, occluder=n >= 8)
    d = b.desc.replace(ref_frame=ref)
    m = b.motion.clone()
    m -= m[ref:ref + 1].clone()
    b = synth.Burst(d, b.tuning, b.frames, m)
    print("[case] stream", n, h, w, scale, tile, cfa, ref, flush=True)
    order = [k for k in range(n) if k != ref]          # hmfsr_merge's visiting order after the base
    got, sm = stream_merge(b, order)
    want = torch_ops.merge(b.frames.to(DEV), b.motion.to(DEV), d, b.tuning)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got, want.cpu().numpy())
    assert sm.state.numel() == 9 * d.out_height * d.out_width   # independent of the frame count
    f, mo = b.numpy()
    assert_parity(got, om.merge(f, mo, d, b.tuning), "stream vs oracle")


def test_stream_other_order_matches_oracle():
    """Any order of the aligned frames merges the same image (eq. 1 is a sum)
    up to float rounding."""
    b = synth.make_burst(6, 96, 96, seed=3200, scale=1.0, tile_size=16)
    got, _ = stream_merge(b, [5, 3, 1, 4, 2])
    f, mo = b.numpy()
    assert_parity(got, om.merge(f, mo, b.desc, b.tuning), "reordered stream vs oracle")
