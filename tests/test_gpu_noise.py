"""Noise model on the GPU (Sec. 5.2.2 Monte-Carlo tables; Sec. 7.2 / S.2
SNR-dependent tuning), through the C ABI, against the oracle.

Tables: the GPU draws the same Philox4x32-10 normals as the oracle and sums
in another order in float64; entries are stored as float32, so they agree to
float32 rounding (relative 1e-6). Merges that read a table meet the forward
tolerance and the adjoint criterion. The SNR comes from an exact integer sum
and the tuning is the same float64 arithmetic: equal bit for bit."""
import numpy as np
import pytest
import torch

import oracle.adjoint as oa
import oracle.merge as om
import oracle.noise as on
from parity_util import assert_parity
from paper_1905_03277_amd import synth, torch_ops
from test_gpu_backward import check, gpu_backward

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("a,b,bins,patches,seed", [(4e-3, 1e-5, 17, 2048, 5), (1e-3, 1e-6, 64, 1000, 2 ** 40 + 3),
                                                   (2e-2, 1e-4, 2, 300, 0)])
def test_table_matches_oracle(a, b, bins, patches, seed):
    print("[case] noise table", a, b, bins, patches, seed, flush=True)
    d = synth.Desc(2, 64, 64, noise_a=a, noise_b=b)
    t = torch_ops.noise_table(d, DEV, bins=bins, patches=patches, seed=seed)
    t2 = torch_ops.noise_table(d, DEV, bins=bins, patches=patches, seed=seed)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.float64)
    assert torch.equal(t, t2)
    want = on.noise_tables(d.noise_a, d.noise_b, d.black_level, d.white_level, bins=bins, patches=patches, seed=seed)
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-15)


def bright_case(n=4, h=48, w=64, scale=1.0, cfa=0, seed=41):
    """Bright, noisy burst: the guide means reach the white point, where the
    table and the closed forms differ."""
    b = synth.make_burst(n, h, w, seed=seed, tile_size=16, scale=scale, cfa=cfa, noise_a=8e-3, noise_b=1e-4)
    f, m = b.numpy()
    f = np.clip(f.astype(np.int64) + 1800, 0, 4095).astype(np.uint16)   # push towards the white point
    d = b.desc
    table = torch_ops.noise_table(d, DEV, bins=33, patches=4096, seed=seed)
    return f, np.ascontiguousarray(m), d.replace(noise_table=table), b.tuning


@pytest.mark.parametrize("case", [dict(), dict(scale=1.5, cfa=2, seed=42), dict(scale=2.0, cfa=1, seed=43, n=3)],
                         ids=["s1", "s15", "s2"])
def test_merge_with_table_matches_oracle(case):
    print("[case] merge with noise table", case, flush=True)
    f, m, d, tun = bright_case(**case)
    out = torch_ops.merge(torch.from_numpy(f.astype(np.int16)).to(DEV), torch.from_numpy(m).to(DEV), d, tun)
    torch.cuda.synchronize()
    want = om.merge(f, m, d, tun)
    assert_parity(out.cpu().numpy(), want, "merge with noise table")
    # and the table matters here
    plain = om.merge(f, m, d.replace(noise_table=None), tun)
    assert np.abs(plain - want).max() > 1e-4


def test_adjoint_with_table():
    f, m, d, tun = bright_case(seed=44)
    rng = np.random.default_rng(3)
    g_out = rng.normal(size=(3, d.out_height, d.out_width)).astype(np.float32)
    want_t, want_m = oa.merge_backward(f, m, d, tun, g_out)
    got_t, got_m = gpu_backward(f, m, d, tun, g_out)
    check(got_t, want_t, "tuning gradient (noise table)")
    check(got_m, want_m, "motion gradient (noise table)")


def test_batch_and_stream_with_table_are_bitwise(monkeypatch):
    monkeypatch.setenv("HMFSR_MERGE_VARIANT", "2")
    f, m, d, tun = bright_case(n=5, seed=45)
    ft = torch.from_numpy(f.astype(np.int16)).to(DEV)
    mt = torch.from_numpy(m).to(DEV)
    one = torch_ops.merge(ft, mt, d, tun)
    (batch,) = torch_ops.merge_batch([(ft, mt, d, tun)])
    sm = torch_ops.StreamingMerge(ft[d.ref_frame].contiguous(), d, tun)
    for k in range(d.n_frames):
        if k != d.ref_frame:
            sm.add(ft[k].contiguous(), mt[k].contiguous())
    stream = sm.result()
    torch.cuda.synchronize()
    assert torch.equal(batch, one)
    assert torch.equal(stream, one)


@pytest.mark.parametrize("noise_a,noise_b,gain", [(1e-3, 1e-6, 1.0), (4e-3, 1e-5, 0.25), (2e-2, 1e-4, 0.05),
                                                  (1e-4, 1e-7, 1.0)])
def test_auto_tuning_matches_oracle_exactly(noise_a, noise_b, gain):
    b = synth.make_burst(3, 96, 128, seed=46, noise_a=noise_a, noise_b=noise_b)
    f, _ = b.numpy()
    f = (64 + (f.astype(np.float64) - 64) * gain).round().astype(np.uint16)   # darker scenes, lower SNR
    d = b.desc.replace(ref_frame=1)
    tun, tile, snr = torch_ops.auto_tuning(torch.from_numpy(f.astype(np.int16)).to(DEV), d)
    want_snr = on.frame_snr(f[1], d.noise_a, d.noise_b, d.black_level, d.white_level)
    want, want_tile = on.snr_tuning(want_snr)
    print("[case] auto tuning", noise_a, noise_b, gain, "snr", snr, flush=True)
    assert snr == want_snr
    assert tile == want_tile
    for k, v in want.items():
        assert getattr(tun, k) == np.float32(v), k
    assert tun.hf_ratio == 0.0
