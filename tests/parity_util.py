"""Helpers for comparing the HIP path with the oracle."""
import math

import numpy as np

import oracle.merge as om

# The forward tolerance on outputs normalised to [0, 1].
MAX_ABS = 2e-4
P999 = 5e-5


def stats(got, want):
    d = np.abs(np.asarray(got, np.float64) - np.asarray(want, np.float64))
    return dict(max=float(d.max()), p999=float(np.quantile(d, 0.999)), mean=float(d.mean()),
                argmax=np.unravel_index(int(d.argmax()), d.shape))


def assert_parity(got, want, what=""):
    st = stats(got, want)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    assert st["max"] <= MAX_ABS and st["p999"] <= P999, f"{what}: {st}"
    return st


def crop_case(frames, motion, desc, oy0, ox0, size_y, size_x, halo=None):
    """Input window (frames, motion, desc) around output rows [oy0, oy0+size_y)
    and columns [ox0, ox0+size_x), plus the index ranges of those output
    pixels in the window's own output grid. The merge is local, so the window's
    interior equals the full image's there as long as the halo covers the
    largest displacement, the 3x3 tile neighbourhood and the robustness
    footprint."""
    n, H, W = frames.shape
    T = desc.tile_size
    s = desc.scale
    if halo is None:
        vmax = float(np.abs(motion).max())
        halo = int(math.ceil((vmax + 2 * T + 16) / 16.0)) * 16
    step = 16 * T // math.gcd(16, T)            # multiple of 16 and of the tile size
    by0 = int(math.floor(oy0 / s))
    bx0 = int(math.floor(ox0 / s))
    by1 = int(math.ceil((oy0 + size_y) / s))
    bx1 = int(math.ceil((ox0 + size_x) / s))
    y0 = max(0, (by0 - halo) // step * step)
    x0 = max(0, (bx0 - halo) // step * step)
    y1 = min(H, by1 + halo)
    x1 = min(W, bx1 + halo)
    y1 += (y1 - y0) & 1
    x1 += (x1 - x0) & 1
    y1, x1 = min(H, y1), min(W, x1)
    # output offset of the window must be integral: y0 * s integer
    assert float(y0 * s).is_integer() and float(x0 * s).is_integer(), (y0, x0, s)
    fr = np.ascontiguousarray(frames[:, y0:y1, x0:x1])
    mo = np.ascontiguousarray(motion[:, y0 // T: -(-y1 // T), x0 // T: -(-x1 // T)])
    d = desc.replace(height=y1 - y0, width=x1 - x0)
    ry = slice(oy0 - int(y0 * s), oy0 - int(y0 * s) + size_y)
    rx = slice(ox0 - int(x0 * s), ox0 - int(x0 * s) + size_x)
    if y1 == H:
        assert d.out_height == desc.out_height - int(y0 * s)
    if x1 == W:
        assert d.out_width == desc.out_width - int(x0 * s)
    return fr, mo, d, ry, rx


def oracle_crop(frames, motion, desc, tuning, oy0, ox0, size_y, size_x):
    fr, mo, d, ry, rx = crop_case(frames, motion, desc, oy0, ox0, size_y, size_x)
    return om.merge_window(fr, mo, d, tuning, ry, rx)
