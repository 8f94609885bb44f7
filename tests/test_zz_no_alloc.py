"""hmfsr_merge_noalloc (the merge with its maps in the library's static
scratch array, no device allocation) through the C ABI: equal bit for bit to
hmfsr_merge on two calls in a row, the second with a smaller burst, and within
the forward tolerance of the oracle; a burst whose maps exceed the scratch is
refused before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import oracle.merge as om
from paper_1905_03277_amd import binding, synth
from parity_util import assert_parity

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def run(entry, b, saved=False):
    """Merge burst b through hmfsr_merge or hmfsr_merge_noalloc (ctypes, the
    C ABI itself); returns the output (and the saved normaliser) on the host."""
    f = b.frames.to(DEV)
    m = b.motion.to(DEV)
    d = b.desc
    out = torch.full((3, d.out_height, d.out_width), float("nan"), dtype=torch.float32, device=DEV)
    sv = torch.zeros((12, d.out_height, d.out_width), dtype=torch.float32, device=DEV) if saved else None
    desc, tun = binding.make_desc(d), binding.make_tuning(b.tuning)
    stream = torch.cuda.current_stream().cuda_stream
    st = getattr(binding.lib(), entry)(ctypes.byref(desc), ctypes.byref(tun), f.data_ptr(), m.data_ptr(),
                                        out.data_ptr(), sv.data_ptr() if saved else None, stream or None)
    assert st == binding.HMFSR_OK, binding.strerror(st)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (sv.cpu().numpy() if saved else None)


def test_noalloc_equals_merge_on_two_calls_second_smaller():
    big = synth.make_burst(8, 512, 640, seed=7100, scale=1.5, tile_size=16, occluder=True)
    small = synth.make_burst(3, 64, 96, seed=7101, scale=2.0, tile_size=8, cfa=2)
    print("[case] noalloc 8x512x640 s1.5 then 3x64x96 s2", flush=True)
    got_big, _ = run("hmfsr_merge_noalloc", big)
    got_small, _ = run("hmfsr_merge_noalloc", small)
    want_big, _ = run("hmfsr_merge", big)
    want_small, _ = run("hmfsr_merge", small)
    np.testing.assert_array_equal(got_big, want_big)
    np.testing.assert_array_equal(got_small, want_small)
    f, m = small.numpy()
    assert_parity(got_small, om.merge(f, m, small.desc, small.tuning), "noalloc small burst")


def test_noalloc_saved_normaliser_and_repeat():
    b = synth.make_burst(5, 96, 128, seed=7200, scale=1.25, tile_size=16, cfa=1)
    print("[case] noalloc with saved", flush=True)
    got, got_sv = run("hmfsr_merge_noalloc", b, saved=True)
    want, want_sv = run("hmfsr_merge", b, saved=True)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(got_sv, want_sv)
    again, _ = run("hmfsr_merge_noalloc", b)
    plain, _ = run("hmfsr_merge", b)
    np.testing.assert_array_equal(again, plain)


def test_noalloc_refuses_bursts_beyond_the_scratch():
    d = synth.Desc(8, 3024, 4032, tile_size=16, scale=1.0)
    desc, tun = binding.make_desc(d), binding.make_tuning(synth.TUNING_SNR22)
    st = binding.lib().hmfsr_merge_noalloc(ctypes.byref(desc), ctypes.byref(tun), 16, 16, 16, None, None)
    assert st == binding.HMFSR_E_TOO_LARGE
    assert "static scratch" in binding.strerror(st)
