"""Pins of the noise-model oracle (Sec. 5.2.2 Monte-Carlo tables; Sec. 7.2 and
supplement S.2 SNR-dependent tuning): the generator against its published
known answers, the simulation against closed forms where they exist, the
table plumbing against the closed-form robustness. No GPU involved."""
import math
import os

import numpy as np
import pytest

import oracle.merge as om
import oracle.noise as on
from paper_1905_03277_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def kat_vectors():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    rows = kat_vectors()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = [int(v) for v in on.philox4x32([np.uint64(c) for c in ctr], key)]
        assert got == want


def test_box_muller_identity_and_moments():
    n = 1 << 17
    ctr = (np.arange(n), np.full(n, 3), np.full(n, 17), np.zeros(n, dtype=np.int64))
    key = (12345, 678)
    w = on.philox4x32(ctr, key)
    u0 = (w[0].astype(np.float64) + 0.5) * 2.0 ** -32
    z = on.normals(ctr, key)
    # the pair's radius is fixed by the first uniform
    np.testing.assert_allclose(z[0] ** 2 + z[1] ** 2, -2.0 * np.log(u0), rtol=1e-12)
    allz = np.concatenate(z)
    se = 1.0 / math.sqrt(allz.size)
    assert abs(allz.mean()) < 5 * se
    assert abs(allz.var() - 1.0) < 5 * math.sqrt(2.0) * se
    assert abs(np.corrcoef(z[0], z[1])[0, 1]) < 5 / math.sqrt(n)
    assert abs(np.corrcoef(z[0], z[2])[0, 1]) < 5 / math.sqrt(n)


def test_unclipped_limit_is_the_closed_form():
    """Far from both ends of the raw range nothing clips: sigma_md^2 -> var and
    d_md^2 -> 2 var / 9 (var halved for the two-green mean)."""
    a, b = 1e-4, 1e-6
    patches = 16384
    t = on.noise_tables(a, b, 64.0, 4095.0, bins=9, patches=patches, seed=7)
    mu = np.arange(9) / 8.0
    var = a * mu + b
    inner = slice(1, 8)          # mu = 1 sits at the white point
    for cls, v in ((0, var), (1, var / 2.0)):
        se_s = v / math.sqrt(8.0 * patches)                 # mean of two unbiased variances
        se_d = (2.0 * v / 9.0) * math.sqrt(2.0 / patches)   # squared normal difference
        assert np.all(np.abs(t[inner, 2 * cls] - v[inner]) < 5 * se_s[inner])
        assert np.all(np.abs(t[inner, 2 * cls + 1] - 2.0 * v[inner] / 9.0) < 5 * se_d[inner])


def test_white_point_clipping_closed_form():
    """At mu = 1 half of the samples clip: var(min(mu + s z, 1)) = s^2 (1/2 -
    1/(2 pi)) for a normal z, 0.34 of the unclipped variance."""
    a, b = 4e-3, 1e-5
    patches = 16384
    t = on.noise_tables(a, b, 64.0, 4095.0, bins=5, patches=patches, seed=11)
    s2 = a * 1.0 + b
    vc = s2 * (0.5 - 1.0 / (2.0 * math.pi))
    assert abs(t[-1, 0] - vc) < 0.05 * vc
    assert abs(t[-1, 1] - 2.0 * vc / 9.0) < 0.08 * (2.0 * vc / 9.0)
    assert abs(t[-1, 2] - vc / 2.0) < 0.05 * vc / 2.0
    # clipping only ever removes variance
    mu = np.arange(5) / 4.0
    assert np.all(t[:, 0] <= (a * mu + b) * 1.05)


def test_table_lookup_interpolates_linearly():
    t = np.zeros((5, 4))
    t[:, 1] = [0.0, 1.0, 4.0, 9.0, 16.0]
    assert on.table_lookup(t, 0.5, 1) == 4.0
    assert on.table_lookup(t, 0.625, 1) == pytest.approx(6.5)
    assert on.table_lookup(t, -0.3, 1) == 0.0
    assert on.table_lookup(t, 1.7, 1) == 16.0
    assert on.table_lookup(t, 1.0, 1) == 16.0


def test_closed_form_table_reproduces_the_closed_form_robustness():
    """The noise variance is linear in brightness, so a table holding the closed
    forms at the bin centres interpolates them exactly (mu in [0, 1]): the merge
    must not change. Pins the table's column layout (R/B vs green)."""
    b = synth.make_burst(4, 48, 64, seed=44, tile_size=16, noise_a=2e-3, noise_b=1e-5)
    f, m = b.numpy()
    bins = 33
    mu = np.arange(bins) / (bins - 1.0)
    var = b.desc.noise_a * mu + b.desc.noise_b
    table = np.stack([var, 2 * var / 9, var / 2, var / 9], axis=1)
    d_tab = b.desc.replace(noise_table=table)
    got = om.merge(f, m, d_tab, b.tuning)
    want = om.merge(f, m, b.desc, b.tuning)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)
    # a table with another model does change it
    d_other = b.desc.replace(noise_table=table * 4.0)
    assert np.abs(om.merge(f, m, d_other, b.tuning) - want).max() > 1e-5


def test_snr_tuning_endpoints_and_steps():
    low, t_low = on.snr_tuning(3.0)
    high, t_high = on.snr_tuning(55.0)
    for k, (lo, hi) in on.RANGES.items():
        assert low[k] == lo and high[k] == hi
    mid, t_mid = on.snr_tuning(18.0)
    for k, (lo, hi) in on.RANGES.items():
        assert mid[k] == pytest.approx(0.5 * (lo + hi), rel=1e-12)
    assert (t_low, on.snr_tuning(13.99)[1], on.snr_tuning(14.0)[1], on.snr_tuning(21.99)[1],
            on.snr_tuning(22.0)[1], t_high) == (64, 64, 32, 32, 16, 16)
    for k, v in on.FIXED.items():
        assert low[k] == v == high[k]
    # monotone: more denoising as the SNR drops
    s = np.linspace(0, 40, 81)
    kd = [on.snr_tuning(x)[0]["k_detail"] for x in s]
    assert np.all(np.diff(kd) <= 0)


def test_frame_snr_of_a_constant_frame():
    f = np.full((8, 10), 64 + 4031 // 4, dtype=np.uint16)     # a quarter of the range
    mu = (4031 // 4) / 4031.0
    want = mu / math.sqrt(1e-3 * mu + 1e-6)
    assert on.frame_snr(f, 1e-3, 1e-6, 64.0, 4095.0) == pytest.approx(want, rel=1e-15)
