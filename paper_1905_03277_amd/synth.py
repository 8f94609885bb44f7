"""Seeded synthetic raw bursts shaped like the paper's workloads.

This module only *draws inputs*: a procedural RGB scene, per-frame handheld
warps, a Bayer mosaic, heteroscedastic noise and 12-bit quantisation, plus the
ground-truth per-tile motion vectors and the tuning sets. It contains none of
the merge arithmetic and is the only module shared by the oracle side
(``oracle/``, tests) and the HIP side (binding, bench).

Recipe (stands in for the paper's real 12 MP Pixel 3 bursts and for its
synthetic Kodak/McMaster bursts, Sec. 6.1, which are not available here):

* Scene, continuous in scene pixels: a base colour U[0.3, 0.7]^3 plus six
  oriented sinusoid gratings (orientation U[0, pi), frequency U[0.02, 0.45]
  cycles/px so the R/B planes alias, phase U[0, 2pi), amplitude U[0.05, 0.2],
  per-channel gains U[0, 1]^3), remapped per channel into [0.05, 0.95] by its
  analytic range, then twelve convex flat-colour polygons (3-7 vertices,
  radius U[0.05, 0.3] * min(H, W), colour U[0.05, 0.95]^3) painted over it.
* Frame n samples the scene by point sampling (the paper's nearest-neighbour
  resampling that keeps aliasing, Sec. 6.1) at Rot(theta_n)(P - ctr) + ctr + t_n
  with t_n ~ N(0, sigma_t^2 I) and theta_n ~ N(0, (0.3 deg)^2).
* Bayer mosaic by CFA, noise x + sqrt(a x + b) N(0, 1) (the heteroscedastic
  model of Sec. 5.2.2), quantised as clip(round(64 + 4031 x), 0, 4095).
* Ground-truth motion per base tile: the clipped tile centre mapped through
  frame 0's warp into the scene and back through frame n's warp.
* Optional occluder: a flat rectangle drawn in frame coordinates in frames
  4-7, moving 20 px per frame (unaligned content the robustness must reject).

Seeds: numpy PCG64 with ``190503277 + 1000 * config + burst`` draws every
scene/warp parameter; a torch generator with the same seed draws the noise.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

CFA_RGGB, CFA_GRBG, CFA_GBRG, CFA_BGGR = 0, 1, 2, 3
# Colour (0=R, 1=G, 2=B) at Bayer parity index (row & 1) * 2 + (col & 1).
_CFA_COLOURS = {
    CFA_RGGB: (0, 1, 1, 2),
    CFA_GRBG: (1, 0, 2, 1),
    CFA_GBRG: (1, 2, 0, 1),
    CFA_BGGR: (2, 1, 1, 0),
}

SEED_BASE = 190503277


def _f32(v) -> float:
    return float(np.float32(v))


@dataclass
class Tuning:
    """Tuning scalars of the merge (supplement S.1/S.2 names)."""
    k_detail: float
    k_denoise: float
    d_th: float
    d_tr: float
    k_stretch: float
    k_shrink: float
    s: float          # paper s_2 (no local motion)
    t: float
    s_motion: float   # paper s_1 (local motion above the threshold)
    m_th: float       # paper M_th, in pixels
    hf_ratio: float = 0.0   # S.3 variance-loss threshold (0: high-frequency rejection off)

    def __post_init__(self):
        # The C ABI carries these as float32: keep the canonical values rounded.
        for f in dataclasses.fields(self):
            setattr(self, f.name, _f32(getattr(self, f.name)))

    def as_list(self):
        return [self.k_detail, self.k_denoise, self.d_th, self.d_tr, self.k_stretch,
                self.k_shrink, self.s, self.t, self.s_motion, self.m_th]

    def replace(self, **kw) -> "Tuning":
        return dataclasses.replace(self, **kw)


# Values inside the printed S.2 ranges, interpolated linearly in SNR over [6, 30]
# (low SNR -> the upper, more denoising end of each range).
TUNING_SNR22 = Tuning(k_detail=0.2755, k_denoise=3.64, d_th=0.00387, d_tr=0.01047,
                      k_stretch=4.0, k_shrink=2.0, s=2.0, t=0.12, s_motion=12.0, m_th=0.8)
TUNING_SNR11 = Tuning(k_detail=0.3128, k_denoise=4.57, d_th=0.00807, d_tr=0.01699,
                      k_stretch=4.0, k_shrink=2.0, s=2.0, t=0.12, s_motion=12.0, m_th=0.8)


@dataclass
class Desc:
    """Burst descriptor (mirrors the C struct ``hmfsr_desc``)."""
    n_frames: int
    height: int
    width: int
    ref_frame: int = 0
    cfa: int = CFA_RGGB
    black_level: float = 64.0
    white_level: float = 4095.0
    noise_a: float = 1e-3
    noise_b: float = 1e-6
    tile_size: int = 16
    scale: float = 1.0
    out_height: int = 0
    out_width: int = 0
    # Monte-Carlo noise table float32 [bins][4] (None: the closed forms); a
    # device tensor for the library, any array for the oracle
    noise_table: object = field(default=None, compare=False, repr=False)

    def __post_init__(self):
        for name in ("black_level", "white_level", "noise_a", "noise_b", "scale"):
            setattr(self, name, _f32(getattr(self, name)))
        if self.out_height == 0:
            self.out_height = int(math.floor(self.height * self.scale + 0.5))
        if self.out_width == 0:
            self.out_width = int(math.floor(self.width * self.scale + 0.5))

    @property
    def tiles_y(self) -> int:
        return -(-self.height // self.tile_size)

    @property
    def tiles_x(self) -> int:
        return -(-self.width // self.tile_size)

    def replace(self, **kw) -> "Desc":
        d = dataclasses.replace(self, **kw)
        if "scale" in kw or "height" in kw or "width" in kw:
            if "out_height" not in kw:
                d.out_height = int(math.floor(d.height * d.scale + 0.5))
            if "out_width" not in kw:
                d.out_width = int(math.floor(d.width * d.scale + 0.5))
        return d


@dataclass
class Burst:
    desc: Desc
    tuning: Tuning
    frames: torch.Tensor            # uint16 [N][H][W]
    motion: torch.Tensor            # float32 [N][TY][TX][2], (vx, vy) in px, motion[ref] = 0
    gt: Optional[torch.Tensor] = None   # float32 [3][OH][OW] scene at output pixel centres
    meta: dict = field(default_factory=dict)

    def to(self, device) -> "Burst":
        return Burst(self.desc, self.tuning, self.frames.to(device), self.motion.to(device),
                     None if self.gt is None else self.gt.to(device), dict(self.meta))

    def numpy(self):
        """(frames uint16, motion float32) as host numpy arrays."""
        return self.frames.cpu().numpy(), self.motion.cpu().numpy()


@dataclass
class SceneParams:
    base: np.ndarray                 # [3]
    g_dir: np.ndarray                # [K][2] unit directions
    g_freq: np.ndarray               # [K]
    g_phase: np.ndarray              # [K]
    g_amp: np.ndarray                # [K]
    g_gain: np.ndarray               # [K][3]
    polys: list                      # list of (vertices [V][2] CCW, colour [3])


def _draw_scene(rng: np.random.Generator, height: int, width: int) -> SceneParams:
    k = 6
    base = rng.uniform(0.3, 0.7, size=3)
    ang = rng.uniform(0.0, math.pi, size=k)
    g_dir = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    g_freq = rng.uniform(0.02, 0.45, size=k)
    g_phase = rng.uniform(0.0, 2 * math.pi, size=k)
    g_amp = rng.uniform(0.05, 0.2, size=k)
    g_gain = rng.uniform(0.0, 1.0, size=(k, 3))
    polys = []
    m = min(height, width)
    for _ in range(12):
        nv = int(rng.integers(3, 8))
        r = rng.uniform(0.05, 0.3) * m
        cx = rng.uniform(0.0, width)
        cy = rng.uniform(0.0, height)
        th = np.sort(rng.uniform(0.0, 2 * math.pi, size=nv))
        verts = np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], axis=1)
        col = rng.uniform(0.05, 0.95, size=3)
        polys.append((verts, col))
    return SceneParams(base, g_dir, g_freq, g_phase, g_amp, g_gain, polys)


def _draw_texture(rng: np.random.Generator, height: int, width: int, k: int = 48,
                  f_lo: float = 0.01, f_hi: float = 0.1) -> SceneParams:
    """Isotropic texture for alignment tests: ``k`` gratings in random
    directions with log-uniform frequencies in [f_lo, f_hi] cycles/px (below
    the half-resolution Nyquist limit, so the 2x2-quad luma is not aliased),
    amplitudes U[0.02, 0.04] and per-channel gains U[0.3, 1]; no polygons."""
    base = rng.uniform(0.3, 0.7, size=3)
    ang = rng.uniform(0.0, math.pi, size=k)
    g_dir = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    g_freq = np.exp(rng.uniform(math.log(f_lo), math.log(f_hi), size=k))
    g_phase = rng.uniform(0.0, 2 * math.pi, size=k)
    g_amp = rng.uniform(0.02, 0.04, size=k)
    g_gain = rng.uniform(0.3, 1.0, size=(k, 3))
    return SceneParams(base, g_dir, g_freq, g_phase, g_amp, g_gain, [])


def eval_scene(sp: SceneParams, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Scene colour at scene points (x, y) -> [3, *x.shape] float64 in [0.05, 0.95]."""
    dt = torch.float64
    dev = x.device
    x = x.to(dt)
    y = y.to(dt)
    out = []
    acc = torch.zeros((len(sp.g_freq),) + tuple(x.shape), dtype=dt, device=dev)
    for i in range(len(sp.g_freq)):
        arg = (2 * math.pi * sp.g_freq[i]) * (x * sp.g_dir[i, 0] + y * sp.g_dir[i, 1]) + sp.g_phase[i]
        acc[i] = sp.g_amp[i] * torch.sin(arg)
    for c in range(3):
        gains = torch.tensor(sp.g_gain[:, c], dtype=dt, device=dev).view(-1, *([1] * x.dim()))
        val = sp.base[c] + (acc * gains).sum(0)
        span = float((sp.g_amp * sp.g_gain[:, c]).sum())
        lo, hi = sp.base[c] - span, sp.base[c] + span
        if hi - lo < 1e-9:
            val = torch.full_like(x, 0.5)
        else:
            val = 0.05 + 0.9 * (val - lo) / (hi - lo)
        out.append(val)
    img = torch.stack(out, 0)
    for verts, col in sp.polys:
        inside = torch.ones_like(x, dtype=torch.bool)
        nv = verts.shape[0]
        for k in range(nv):
            ax, ay = verts[k]
            bx, by = verts[(k + 1) % nv]
            cross = (bx - ax) * (y - ay) - (by - ay) * (x - ax)
            inside &= cross >= 0
        for c in range(3):
            img[c] = torch.where(inside, torch.full_like(x, col[c]), img[c])
    return img


def _warp(points_x, points_y, theta, tx, ty, cx, cy):
    """Frame-pixel point -> scene point: Rot(theta)(P - ctr) + ctr + t."""
    c, s = math.cos(theta), math.sin(theta)
    dx, dy = points_x - cx, points_y - cy
    return c * dx - s * dy + cx + tx, s * dx + c * dy + cy + ty


def _unwarp(sx, sy, theta, tx, ty, cx, cy):
    """Scene point -> frame-pixel point (inverse of ``_warp``)."""
    c, s = math.cos(theta), math.sin(theta)
    dx, dy = sx - cx - tx, sy - cy - ty
    return c * dx + s * dy + cx, -s * dx + c * dy + cy


def make_burst(n_frames: int, height: int, width: int, *, seed: int, sigma_t: float = 1.5,
               rot_sigma_deg: float = 0.3, noise_a: float = 1e-3, noise_b: float = 1e-6,
               scale: float = 1.0, tile_size: int = 16, cfa: int = CFA_RGGB,
               tuning: Tuning = TUNING_SNR22, occluder: bool = False, with_gt: bool = False,
               scene: str = "default",
               device="cpu", rows_per_chunk: int = 512) -> Burst:
    """Draw one seeded burst. Frames are generated on ``device`` in row chunks."""
    assert height % 2 == 0 and width % 2 == 0
    rng = np.random.Generator(np.random.PCG64(seed))
    if scene == "default":
        sp = _draw_scene(rng, height, width)
    elif scene == "texture":
        sp = _draw_texture(rng, height, width)
    else:
        raise ValueError(f"unknown scene {scene!r}")
    thetas = rng.normal(0.0, math.radians(rot_sigma_deg), size=n_frames)
    trans = rng.normal(0.0, sigma_t, size=(n_frames, 2))
    occ = None
    if occluder:
        ow, oh = min(400, width // 2), min(300, height // 2)
        x0 = rng.uniform(0.0, max(1.0, width - ow - 20 * 4))
        y0 = rng.uniform(0.0, max(1.0, height - oh))
        occ = (x0, y0, ow, oh, rng.uniform(0.05, 0.95, size=3))
    cx, cy = width / 2.0, height / 2.0
    colours = _CFA_COLOURS[cfa]

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    frames = torch.empty((n_frames, height, width), dtype=torch.int32, device=device)
    cols = torch.arange(width, dtype=torch.float64, device=device) + 0.5
    ch_col = torch.tensor(colours, dtype=torch.int64, device=device)
    for n in range(n_frames):
        for r0 in range(0, height, rows_per_chunk):
            r1 = min(height, r0 + rows_per_chunk)
            rows = torch.arange(r0, r1, dtype=torch.float64, device=device) + 0.5
            py, px = torch.meshgrid(rows, cols, indexing="ij")
            sx, sy = _warp(px, py, thetas[n], trans[n, 0], trans[n, 1], cx, cy)
            rgb = eval_scene(sp, sx, sy)
            if occ is not None and 4 <= n <= 7:
                ox0 = occ[0] + 20.0 * (n - 4)
                inside = (px >= ox0) & (px < ox0 + occ[2]) & (py >= occ[1]) & (py < occ[1] + occ[3])
                for c in range(3):
                    rgb[c] = torch.where(inside, torch.full_like(px, occ[4][c]), rgb[c])
            ri = torch.arange(r0, r1, device=device).view(-1, 1) & 1
            ci = torch.arange(width, device=device).view(1, -1) & 1
            chan = ch_col[ri * 2 + ci]
            x = torch.gather(rgb, 0, chan.unsqueeze(0)).squeeze(0)
            sd = torch.sqrt(torch.clamp(noise_a * x + noise_b, min=0.0))
            z = torch.randn(x.shape, generator=gen, dtype=torch.float64, device=device)
            q = torch.clamp(torch.round(64.0 + 4031.0 * (x + sd * z)), 0, 4095)
            frames[n, r0:r1] = q.to(torch.int32)

    desc = Desc(n_frames=n_frames, height=height, width=width, ref_frame=0, cfa=cfa,
                noise_a=noise_a, noise_b=noise_b, tile_size=tile_size, scale=scale)
    ty_n, tx_n = desc.tiles_y, desc.tiles_x
    tcx = (np.minimum((np.arange(tx_n) + 1) * tile_size, width) + np.arange(tx_n) * tile_size) / 2.0
    tcy = (np.minimum((np.arange(ty_n) + 1) * tile_size, height) + np.arange(ty_n) * tile_size) / 2.0
    gy, gx = np.meshgrid(tcy, tcx, indexing="ij")
    motion = np.zeros((n_frames, ty_n, tx_n, 2), dtype=np.float32)
    sx, sy = _warp(gx, gy, thetas[0], trans[0, 0], trans[0, 1], cx, cy)
    for n in range(n_frames):
        if n == desc.ref_frame:
            continue
        pxn, pyn = _unwarp(sx, sy, thetas[n], trans[n, 0], trans[n, 1], cx, cy)
        motion[n, :, :, 0] = (pxn - gx).astype(np.float32)
        motion[n, :, :, 1] = (pyn - gy).astype(np.float32)

    gt = None
    if with_gt:
        oh_, ow_ = desc.out_height, desc.out_width
        gt = torch.empty((3, oh_, ow_), dtype=torch.float32, device=device)
        ocols = (torch.arange(ow_, dtype=torch.float64, device=device) + 0.5) / scale
        for r0 in range(0, oh_, rows_per_chunk):
            r1 = min(oh_, r0 + rows_per_chunk)
            orows = (torch.arange(r0, r1, dtype=torch.float64, device=device) + 0.5) / scale
            py, px = torch.meshgrid(orows, ocols, indexing="ij")
            sx0, sy0 = _warp(px, py, thetas[0], trans[0, 0], trans[0, 1], cx, cy)
            gt[:, r0:r1] = eval_scene(sp, sx0, sy0).to(torch.float32)

    frames_t = None
    if str(device) != "cpu":
        try:  # convert on the device when torch supports it
            frames_t = frames.to(torch.uint16)
        except (RuntimeError, TypeError):
            frames_t = None
    if frames_t is None:
        frames_t = torch.from_numpy(frames.cpu().numpy().astype(np.uint16))
        if str(device) != "cpu":
            frames_t = frames_t.to(device)
    del frames
    meta = {"seed": seed, "thetas": thetas, "trans": trans, "occluder": occ}
    return Burst(desc, tuning, frames_t, torch.from_numpy(motion).to(device), gt, meta)


# --- the five workloads -------------------------------------------------------

def config_seed(config: int, burst: int = 0) -> int:
    return SEED_BASE + 1000 * config + burst


def make_config(config: int, burst: int = 0, device="cpu", **over) -> Burst:
    """Burst for workload 1 (8x256x256), 2 (8x3024x4032 + occluder),
    3 (15x1512x2016 low light, scale 2) or 5 (8x768x1024, scale 2, with GT)."""
    seed = config_seed(config, burst)
    if config == 1:
        kw = dict(n_frames=8, height=256, width=256, sigma_t=1.5, noise_a=1e-3, noise_b=1e-6,
                  scale=1.0, tuning=TUNING_SNR22)
    elif config == 2:
        kw = dict(n_frames=8, height=3024, width=4032, sigma_t=1.5, noise_a=1e-3, noise_b=1e-6,
                  scale=1.0, tuning=TUNING_SNR22, occluder=True)
    elif config == 3:
        kw = dict(n_frames=15, height=1512, width=2016, sigma_t=2.0, noise_a=4e-3, noise_b=1e-5,
                  scale=2.0, tuning=TUNING_SNR11)
    elif config == 5:
        kw = dict(n_frames=8, height=768, width=1024, sigma_t=1.5, noise_a=1e-3, noise_b=1e-6,
                  scale=2.0, tuning=TUNING_SNR22, with_gt=True)
    else:
        raise ValueError(f"no single-burst workload {config}")
    kw.update(over)
    return make_burst(seed=seed, device=device, **kw)


BATCH_SIZES = [(384, 512), (768, 1024), (1512, 2016), (3024, 4032)]   # (H, W)
BATCH_SCALES = [1.0, 1.5, 2.0]


def batch_plan(n_bursts: int = 64, seed: int = SEED_BASE + 4000):
    """(n_frames, H, W, scale) per burst of the uneven batched workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    plan = []
    for _ in range(n_bursts):
        n = int(rng.integers(2, 16))
        h, w = BATCH_SIZES[int(rng.integers(0, len(BATCH_SIZES)))]
        s = BATCH_SCALES[int(rng.integers(0, len(BATCH_SCALES)))]
        plan.append((n, h, w, s))
    return plan


def make_batch(n_bursts: int = 64, device="cpu", size_cap=None) -> list:
    """The uneven batched workload: frame count U{2..15}, size and scale drawn
    from fixed lists. ``size_cap`` = (H, W) limits sizes for small test runs."""
    out = []
    for i, (n, h, w, s) in enumerate(batch_plan(n_bursts)):
        if size_cap is not None:
            h, w = min(h, size_cap[0]), min(w, size_cap[1])
        out.append(make_burst(n, h, w, seed=config_seed(4, i), scale=s, device=device))
    return out
