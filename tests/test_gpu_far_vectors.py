"""Displacements that throw whole tiles far outside the frame (+-200 and
+-400 px, and beyond the kernels' clamp), against the oracle: the forward of
every compiled tile shape, the robustness maps and the adjoint. Pixels whose
nine samples all leave the frame get no term from that frame (eq. 1 sums over
in-frame samples), and the LDS windows of a tile stop at the frame's ring."""
import numpy as np
import pytest
import torch

import oracle.adjoint as oa
import oracle.merge as om
from paper_1905_03277_amd import synth, torch_ops
from parity_util import assert_parity
from test_gpu_backward import check, gpu_backward

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def far_field(m, rng, jumps=(200.0, -200.0, 400.0, -400.0)):
    """The generator's field with the edge tiles of every aligned frame thrown
    out by +-200 / +-400 px (each frame another edge and axis) and a few
    interior tiles jumping by the same amounts."""
    m = m.copy()
    n, ty, tx, _ = m.shape
    for k in range(1, n):
        j = jumps[(k - 1) % len(jumps)]
        side = (k - 1) % 4
        if side == 0:
            m[k, :, tx - 1, 0] += j        # right column, horizontally
        elif side == 1:
            m[k, ty - 1, :, 1] += j        # bottom row, vertically
        elif side == 2:
            m[k, :, 0, 0] += j             # left column
        else:
            m[k, 0, :, 1] += j             # top row
        for _ in range(3):
            m[k, rng.integers(0, ty), rng.integers(0, tx), rng.integers(0, 2)] += jumps[rng.integers(0, 4)]
    m[0] = 0
    return m.astype(np.float32)


def gpu_merge(f, m, desc, tuning):
    out = torch_ops.merge(torch.from_numpy(f.astype(np.int16)).to(DEV), torch.from_numpy(m).to(DEV), desc, tuning)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("scale", [1.0, 1.5])
def test_forward_far_vectors(variant, scale, monkeypatch):
    monkeypatch.setenv("HMFSR_MERGE_VARIANT", str(variant))
    b = synth.make_burst(5, 256, 256, seed=4100 + variant, scale=scale, tile_size=16)
    f, m = b.numpy()
    m = far_field(m, np.random.default_rng(4200 + variant))
    print(f"[case] far vectors variant {variant} scale {scale}", flush=True)
    assert_parity(gpu_merge(f, m, b.desc, b.tuning), om.merge(f, m, b.desc, b.tuning), "far vectors")


def test_forward_vectors_beyond_the_clamp():
    """Vectors of 1e6 px and infinities: the kernels clamp them to just past
    the frame, where no sample is in the frame, which changes no result; the
    oracle sees no in-frame sample either."""
    b = synth.make_burst(4, 64, 96, seed=4300, scale=1.5, tile_size=16)
    f, m = b.numpy()
    m = m.copy()
    m[1, 1, 2] = (1e6, -1e6)
    m[2, 0, :, 0] = np.inf
    m[3, 2, 3, 1] = -np.inf
    m = m.astype(np.float32)
    mo = np.where(np.isfinite(m), m, np.sign(m) * 1e6).astype(np.float32)  # the oracle takes finite values
    print("[case] vectors beyond the clamp", flush=True)
    assert_parity(gpu_merge(f, m, b.desc, b.tuning), om.merge(f, mo, b.desc, b.tuning), "beyond the clamp")


def test_robustness_maps_far_vectors():
    b = synth.make_burst(5, 128, 192, seed=4400, scale=1.0, tile_size=16)
    f, m = b.numpy()
    m = far_field(m, np.random.default_rng(4401))
    print("[case] robustness maps, far vectors", flush=True)
    maps = torch_ops.merge_maps(torch.from_numpy(f.astype(np.int16)).to(DEV), torch.from_numpy(m).to(DEV),
                                b.desc, b.tuning)
    ref = om.prepare(f, m, b.desc, b.tuning)
    np.testing.assert_allclose(maps["robust"].cpu().numpy(), ref["r"], rtol=0, atol=5e-5)
    np.testing.assert_allclose(maps["robust_min"].cpu().numpy(), ref["r_hat"], rtol=0, atol=5e-5)


@pytest.mark.parametrize("scale", [1.0, 2.0])
def test_adjoint_far_vectors(scale):
    b = synth.make_burst(5, 96, 160, seed=4500, scale=scale, tile_size=16)
    f, m = b.numpy()
    rng = np.random.default_rng(4501)
    m = far_field(m + (np.round(rng.normal(0, 0.1, m.shape) * 64) / 64).astype(np.float32), rng)
    g_out = rng.normal(size=(3, b.desc.out_height, b.desc.out_width)).astype(np.float32)
    print(f"[case] adjoint far vectors scale {scale}", flush=True)
    want_t, want_m = oa.merge_backward(f, m, b.desc, b.tuning, g_out)
    got_t, got_m = gpu_backward(f, m, b.desc, b.tuning, g_out)
    check(got_t, want_t, "tuning gradient")
    check(got_m, want_m, "motion gradient")
