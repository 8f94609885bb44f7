"""Pins of the high-frequency artefact rejection (supplement S.3) in the
oracle: the variance-loss test against closed forms, and its effect on the
robustness (full rejection only where the loss meets a strongly varying
vector field). No GPU involved."""
import numpy as np
import pytest

import oracle.merge as om
from brute_twin import brute_merge
from paper_1905_03277_amd import synth

TUN = synth.TUNING_SNR22


def quad_frame(v):
    """Raw frame whose 2x2 quads are uniform with half-res values v [h][w]."""
    v = np.asarray(v, dtype=np.int64)
    return np.repeat(np.repeat(v, 2, axis=0), 2, axis=1).astype(np.uint16)


def interior(m, k=2):
    return m[k:-k, k:-k]


@pytest.mark.parametrize("cfa", [0, 3])
def test_checkerboard_loses_all_but_one_81st(cfa):
    """A half-res checkerboard: 3x3 windows hold 5 of one value and 4 of the
    other, so the variance before is 20/81 of the squared step and the box
    means alternate by a ninth of the step: the variance after is exactly
    1/81 of the variance before. The test fires for ratios above 1/81 only."""
    h, w = 12, 14
    ii, jj = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    f = quad_frame(1000 + 500 * ((ii + jj) % 2))
    assert interior(om.variance_loss(f, cfa, 1.0 / 81.0 + 1e-6)).all()
    assert not interior(om.variance_loss(f, cfa, 1.0 / 81.0 - 1e-6)).any()


def test_ramp_keeps_its_variance():
    """A linear ramp is its own 3x3 mean: the variance after equals the
    variance before (ratio 1) away from the edges."""
    h, w = 10, 16
    _, jj = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    f = quad_frame(1000 + 7 * jj)
    assert not interior(om.variance_loss(f, 0, 1.0)).any()
    assert interior(om.variance_loss(f, 0, 1.0001)).all()


def test_flat_and_disabled():
    f = quad_frame(np.full((8, 8), 1234))
    assert not om.variance_loss(f, 0, 0.5).any()          # no variance at all
    rng = np.random.default_rng(4)
    g = rng.integers(0, 4096, size=(16, 16)).astype(np.uint16)
    assert not om.variance_loss(g, 0, 0.0).any()           # 0 disables


def test_white_noise_against_a_noisy_chart():
    """Noise is high-frequency too: the variance its 3x3 means keep has a
    median near 6 % (a wide spread), while a checker chart keeps 1/81. At a
    threshold of 0.02 the chart is flagged almost everywhere and noise rarely."""
    rng = np.random.default_rng(5)
    f = quad_frame(rng.integers(1000, 3000, size=(96, 96)))
    assert interior(om.variance_loss(f, 0, 0.02)).mean() < 0.1
    assert interior(om.variance_loss(f, 0, 0.2)).mean() > 0.95
    ii, jj = np.meshgrid(np.arange(96), np.arange(96), indexing="ij")
    g = quad_frame(2000 + 600 * ((ii + jj) % 2) + rng.integers(-100, 100, size=(96, 96)))
    assert interior(om.variance_loss(g, 0, 0.02)).mean() > 0.9


def chart_burst(hf_ratio, seed=21, n=4, size=32, tile=8):
    """A small burst whose base frame carries a high-frequency checker patch
    (a test chart) and whose frame 2 has a corrupted tile inside it."""
    b = synth.make_burst(n, size, size, seed=seed, tile_size=tile, sigma_t=1.0)
    f, m = b.numpy()
    f = f.copy()
    m = m.copy()
    hh = size // 2
    ii, jj = np.meshgrid(np.arange(hh), np.arange(hh), indexing="ij")
    patch = quad_frame(900 + 1800 * ((ii + jj) % 2))
    f[b.desc.ref_frame, :size // 2 + 8, :size // 2 + 8] = patch[:size // 2 + 8, :size // 2 + 8]
    m[2, 1, 1] += np.float32(2.5)           # strong local variation: tiles around (1, 1) "move"
    return f, m, b.desc, TUN.replace(hf_ratio=hf_ratio)


def test_rejection_only_where_loss_meets_motion():
    f, m, d, tun = chart_burst(0.05)
    maps = om.prepare(f, m, d, tun)
    base = om.prepare(f, m, d, TUN)
    rej = maps["hf_reject"]
    loss = om.variance_loss(f[d.ref_frame], d.cfa, 0.05)
    assert rej[2].any() and loss.any()
    moving, _ = om.motion_prior(m[2], 1.0, 0.0, tun.m_th)
    h, w = loss.shape
    ii, jj = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    mov_px = moving[np.minimum(2 * ii // d.tile_size, moving.shape[0] - 1),
                    np.minimum(2 * jj // d.tile_size, moving.shape[1] - 1)] > 0.5
    np.testing.assert_array_equal(rej[2], loss & mov_px)
    assert np.all(maps["r"][2][rej[2]] == 0.0)
    np.testing.assert_array_equal(maps["r"][2][~rej[2]], base["r"][2][~rej[2]])
    assert not rej[d.ref_frame].any()
    # frames whose tiles do not move are untouched
    for k in (1, 3):
        if not rej[k].any():
            np.testing.assert_array_equal(maps["r"][k], base["r"][k])


def test_zero_ratio_changes_nothing():
    f, m, d, _ = chart_burst(0.0)
    np.testing.assert_array_equal(om.merge(f, m, d, TUN.replace(hf_ratio=0.0)), om.merge(f, m, d, TUN))


@pytest.mark.parametrize("scale", [1.0, 1.5])
def test_brute_force_twin_with_rejection(scale):
    f, m, d, tun = chart_burst(0.05)
    d = d.replace(scale=scale)
    maps = om.prepare(f, m, d, tun)
    assert maps["hf_reject"].any()
    got = om.merge(f, m, d, tun)
    want = np.array(brute_merge(f.tolist(), m.tolist(), d, tun))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11)
    # and the rejection changes the result
    assert np.abs(got - om.merge(f, m, d, TUN)).max() > 1e-4
