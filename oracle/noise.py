"""FP64 CPU oracle of the noise-model tables and the SNR-dependent tuning.

TEST INFRASTRUCTURE ONLY, like ``oracle/merge.py``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU baseline leg of ``bench.py`` may use it.

Sec. 5.2.2 obtains the modelled spatial standard deviation sigma_md and the
modelled difference of means d_md by Monte-Carlo simulation of constant
patches per brightness level, so that sensor clipping near the white point is
accounted for; eq. (6) then uses them. Sec. 7.2 and supplement S.2 make the
tuning scalars piecewise-linear functions of the base frame's SNR over
[6, 30], with the SNR computed from the mean brightness and the noise model.
Neither the simulation nor the breakpoints are specified further; the
readings below fill them in and are shared with the device code.

Readings (Monte-Carlo tables):
  * random numbers: Philox4x32-10 (Salmon et al., SC 2011), counter
    (patch, bin, 16 * class + j, 0), key (seed mod 2^32, seed div 2^32); each
    call gives four uint32 u, mapped to (u + 1/2) 2^-32 and paired by
    Box-Muller (z = sqrt(-2 ln u_a) cos / sin (2 pi u_b)) into four normals,
    normal q of a patch taken from call j = q // 4;
  * brightness bins mu_i = i / (bins - 1), i = 0 .. bins - 1 (normalised units);
  * a raw sample is mu + sqrt(a max(mu, 0) + b) z, clipped to the raw range
    [-black / (white - black), 1];
  * class 0 (R or B guide pixel): one sample per guide pixel; class 1 (the
    guide's green): the mean of two samples;
  * per patch, two frames of nine guide pixels (normal q = ((frame * 9) +
    pixel) * k + sub, k = 1 or 2 samples per guide pixel);
  * sigma_md^2 = mean over patches of the two frames' unbiased sample
    variances; d_md^2 = mean over patches of the squared difference of the
    two frames' means (both converge to var and 2 var / 9, the closed forms,
    where nothing clips);
  * table layout float [bins][4]: (sigma_md^2, d_md^2) of class 0, then of
    class 1; lookup by linear interpolation at clamp(mu, 0, 1) (bins - 1).

Readings (SNR-dependent tuning):
  * SNR = mu / sqrt(a max(mu, 0) + b), mu the mean of the base frame's
    normalised raw values (its integer sum divided by the pixel count);
  * with s = clamp((SNR - 6) / 24, 0, 1): k_detail 0.33 -> 0.25, k_denoise
    5.0 -> 3.0, D_th 0.010 -> 0.001, D_tr 0.020 -> 0.006 as v = (1 - s) v_low +
    s v_high (exact at both ends; low SNR denoises more); the others fixed at
    S.2's values (k_stretch 4, k_shrink 2, t 0.12, s1 12, s2 2, M_th 0.8 px);
  * tile size T_s = 64 below SNR 14, 32 below SNR 22, else 16.
"""
from __future__ import annotations

import numpy as np

PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


# --------------------------------------------------------------------------- #
# Philox4x32-10                                                               #
# --------------------------------------------------------------------------- #
def philox4x32(ctr, key, rounds=10):
    """Philox4x32 on arrays: ctr = 4 arrays of 32-bit values, key = 2 values.
    Returns 4 uint64 arrays holding 32-bit words."""
    c = [np.asarray(v, dtype=np.uint64) & _MASK for v in ctr]
    k0, k1 = np.uint64(key[0]) & _MASK, np.uint64(key[1]) & _MASK
    m0, m1 = np.uint64(PHILOX_M[0]), np.uint64(PHILOX_M[1])
    for r in range(rounds):
        if r:
            k0 = (k0 + np.uint64(PHILOX_W[0])) & _MASK
            k1 = (k1 + np.uint64(PHILOX_W[1])) & _MASK
        p0 = m0 * c[0]                 # < 2^64: exact in uint64
        p1 = m1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & _MASK, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & _MASK]
    return c


def normals(ctr, key):
    """Four standard normals per counter (Box-Muller on the four uniforms)."""
    u = [(w.astype(np.float64) + 0.5) * 2.0 ** -32 for w in philox4x32(ctr, key)]
    r0 = np.sqrt(-2.0 * np.log(u[0]))
    r1 = np.sqrt(-2.0 * np.log(u[2]))
    t0 = 2.0 * np.pi * u[1]
    t1 = 2.0 * np.pi * u[3]
    return r0 * np.cos(t0), r0 * np.sin(t0), r1 * np.cos(t1), r1 * np.sin(t1)


# --------------------------------------------------------------------------- #
# Monte-Carlo tables of sigma_md^2 and d_md^2                                 #
# --------------------------------------------------------------------------- #
def noise_tables(noise_a, noise_b, black, white, bins=64, patches=4096, seed=0):
    """Table float64 [bins][4]: (sigma_md^2, d_md^2) for the R/B guide pixel,
    then for the two-green mean, per brightness bin (normalised units)."""
    a, b = float(noise_a), float(noise_b)
    lo = -float(black) / (float(white) - float(black))
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    out = np.zeros((bins, 4))
    p_idx, b_idx = np.meshgrid(np.arange(patches), np.arange(bins), indexing="ij")   # [P][bins]
    mu = b_idx / (bins - 1.0)
    sd = np.sqrt(a * np.maximum(mu, 0.0) + b)
    for cls, k in ((0, 1), (1, 2)):
        nq = 2 * 9 * k
        z = []
        for j in range((nq + 3) // 4):
            z.extend(normals((p_idx, b_idx, np.full_like(p_idx, 16 * cls + j), np.zeros_like(p_idx)), key))
        z = np.stack(z[:nq])                                      # [nq][P][bins]
        x = np.clip(mu + sd * z, lo, 1.0)
        g = x.reshape(2, 9, k, patches, bins).mean(axis=2)       # [frame][pixel][P][bins]
        m = g.mean(axis=1)                                        # [frame][P][bins]
        var = ((g - m[:, None]) ** 2).sum(axis=1) / 8.0           # unbiased, [frame][P][bins]
        out[:, 2 * cls] = (0.5 * (var[0] + var[1])).mean(axis=0)
        out[:, 2 * cls + 1] = ((m[0] - m[1]) ** 2).mean(axis=0)
    return out


def table_lookup(table, mu, col):
    """Linear interpolation of table[:, col] at brightness mu (normalised)."""
    t = np.asarray(table, dtype=np.float64)
    bins = t.shape[0]
    x = np.clip(np.asarray(mu, dtype=np.float64), 0.0, 1.0) * (bins - 1)
    i = np.minimum(np.floor(x).astype(np.int64), bins - 2)
    f = x - i
    return (1.0 - f) * t[i, col] + f * t[i + 1, col]


# --------------------------------------------------------------------------- #
# SNR-dependent tuning                                                        #
# --------------------------------------------------------------------------- #
SNR_LOW, SNR_HIGH = 6.0, 30.0
RANGES = {"k_detail": (0.33, 0.25), "k_denoise": (5.0, 3.0), "d_th": (0.010, 0.001), "d_tr": (0.020, 0.006)}
FIXED = {"k_stretch": 4.0, "k_shrink": 2.0, "s": 2.0, "t": 0.12, "s_motion": 12.0, "m_th": 0.8}


def frame_snr(frame, noise_a, noise_b, black, white):
    """SNR of a frame at its mean brightness under the noise model."""
    f = np.asarray(frame)
    mean_raw = int(f.astype(np.int64).sum()) / float(f.size)
    mu = (mean_raw - float(black)) / (float(white) - float(black))
    return mu / np.sqrt(float(noise_a) * max(mu, 0.0) + float(noise_b))


def snr_tuning(snr):
    """(tuning dict, tile size) for a base-frame SNR."""
    s = min(max((float(snr) - SNR_LOW) / (SNR_HIGH - SNR_LOW), 0.0), 1.0)
    tun = {k: (1.0 - s) * lo + s * hi for k, (lo, hi) in RANGES.items()}
    tun.update(FIXED)
    tile = 64 if snr < 14.0 else (32 if snr < 22.0 else 16)
    return tun, tile
