"""FP64 CPU oracle of the kernel-regression burst merge.

TEST INFRASTRUCTURE ONLY. This module is the plain, slow reference the HIP path
is checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it; the product path never does.

It follows Wronski et al., "Handheld Multi-Frame Super-Resolution" (ACM TOG
38(4), 2019), Sec. 5 and supplement S.1, step by step, in float64 numpy, and
shares no code with the HIP side. Steps, in the paper's order:

  1. raw CFA samples -> normalised values               (Sec. 5.1, raw input)
  2. half-resolution luma from 2x2 Bayer quads           (Sec. 5.1.2)
     and the half-resolution RGB guide image             (Sec. 5.2.2)
  3. gradient structure tensor, eq. (3)                  (Sec. 5.1.2)
  4. eigen-analysis -> kernel covariance Omega, eq. (4),
     with the S.1 heuristics A, D, k1^, k2^, k1, k2      (Sec. 5.1.2, S.1)
  5. guide 3x3 colour mean / spatial sigma               (Sec. 5.2.2)
  6. motion prior M per tile, eqs. (7)-(8)               (Sec. 5.2.3)
  7. noise-corrected robustness R, eqs. (5)-(6),
     refined by the 5x5 minimum, eq. (9)                 (Sec. 5.2.1-5.2.3)
  8. per output pixel and frame: nine nearest samples,
     anisotropic Gaussian weights, eq. (2)               (Sec. 5.1, 5.1.1)
  9. per-channel normalised accumulation, eq. (1)        (Sec. 5.1)

Where the paper leaves a point open, the reading taken is stated in the
docstring of the step that implements it.

Coordinates are "edge" coordinates of the full-resolution Bayer grid: pixel
(r, c) covers [c, c+1) x [r, r+1) and has its centre at (c + 1/2, r + 1/2).
Half-resolution pixel (I, J) covers Bayer rows 2I..2I+1, columns 2J..2J+1 and
is centred at (2J + 1, 2I + 1); a full-resolution edge coordinate P maps to the
continuous half-resolution index P / 2 - 1/2. Half-resolution maps are
extended by clamping to the edge.
"""
from __future__ import annotations

import numpy as np

# Colour (0 = R, 1 = G, 2 = B) of Bayer parity index (row & 1) * 2 + (col & 1)
# for the four standard 2x2 mosaics, in the order RGGB, GRBG, GBRG, BGGR.
BAYER_COLOURS = {
    0: (0, 1, 1, 2),
    1: (1, 0, 2, 1),
    2: (1, 2, 0, 1),
    3: (2, 1, 1, 0),
}


def _get(obj, name):
    return obj[name] if isinstance(obj, dict) else getattr(obj, name)


def _opt(obj, name, default):
    """Optional tuning value (absent in older tuning sets)."""
    if isinstance(obj, dict):
        return obj.get(name, default)
    return getattr(obj, name, default)


# --------------------------------------------------------------------------- #
# step 1: normalisation                                                       #
# --------------------------------------------------------------------------- #
def normalise(frames, black, white):
    """x = (raw - black) / (white - black), float64, not clamped."""
    return (np.asarray(frames, dtype=np.float64) - float(black)) / (float(white) - float(black))


def colour_map(height, width, cfa):
    """[H][W] colour index of every Bayer pixel."""
    table = np.array(BAYER_COLOURS[int(cfa)])
    r = np.arange(height)[:, None] & 1
    c = np.arange(width)[None, :] & 1
    return table[r * 2 + c]


# --------------------------------------------------------------------------- #
# step 2: half-resolution luma and guide                                      #
# --------------------------------------------------------------------------- #
def halfres_luma(x):
    """Luma of every 2x2 quad: the mean of its four values (Sec. 5.1.2). x: [..., H, W]."""
    q = x.reshape(x.shape[:-2] + (x.shape[-2] // 2, 2, x.shape[-1] // 2, 2))
    return (q[..., 0, :, 0] + q[..., 0, :, 1] + q[..., 1, :, 0] + q[..., 1, :, 1]) / 4.0


def halfres_guide(x, cfa):
    """Guide RGB per quad: R and B taken directly, the two greens averaged (Sec. 5.2.2).
    x: [..., H, W] -> [..., 3, H/2, W/2]."""
    table = BAYER_COLOURS[int(cfa)]
    q = x.reshape(x.shape[:-2] + (x.shape[-2] // 2, 2, x.shape[-1] // 2, 2))
    pos = {(pr, pc): q[..., pr, :, pc] for pr in (0, 1) for pc in (0, 1)}
    red = [pos[(k >> 1, k & 1)] for k in range(4) if table[k] == 0]
    green = [pos[(k >> 1, k & 1)] for k in range(4) if table[k] == 1]
    blue = [pos[(k >> 1, k & 1)] for k in range(4) if table[k] == 2]
    assert len(red) == 1 and len(green) == 2 and len(blue) == 1
    return np.stack([red[0], (green[0] + green[1]) / 2.0, blue[0]], axis=-3)


# --------------------------------------------------------------------------- #
# step 3: structure tensor                                                    #
# --------------------------------------------------------------------------- #
def structure_tensor(lum):
    """Gradient structure tensor of eq. (3) per half-resolution pixel.

    Reading: the 3x3 luma window around (I, J) holds four 2x2 cells; each cell
    gives one forward-difference gradient (horizontal and vertical differences
    averaged over the cell's two rows / columns). The tensor is the mean of the
    four outer products g g^T. Returns (Ixx, Ixy, Iyy), each [..., h, w]."""
    pad = [(0, 0)] * (lum.ndim - 2) + [(1, 1), (1, 1)]
    lp = np.pad(lum, pad, mode="edge")
    a = lp[..., :-1, :-1]
    b = lp[..., :-1, 1:]
    c = lp[..., 1:, :-1]
    d = lp[..., 1:, 1:]
    gx = ((b - a) + (d - c)) / 2.0          # cell gradients, [..., h+1, w+1]
    gy = ((c - a) + (d - b)) / 2.0
    xx, xy, yy = gx * gx, gx * gy, gy * gy

    def four_cells(m):
        return (m[..., :-1, :-1] + m[..., :-1, 1:] + m[..., 1:, :-1] + m[..., 1:, 1:]) / 4.0

    return four_cells(xx), four_cells(xy), four_cells(yy)


# --------------------------------------------------------------------------- #
# step 4: kernel covariance                                                   #
# --------------------------------------------------------------------------- #
def kernel_covariance(ixx, ixy, iyy, tuning, return_parts=False):
    """Omega of eq. (4) from the eigen-analysis of the structure tensor and the
    heuristics of supplement S.1.

    Readings: the dominant eigenvector e1 (eigenvalue lambda1) points along the
    gradient; the stretched variance k1 is applied along the edge (orthogonal
    to e1) and k2 along the gradient, as the paper's text and figures describe.
    A = 1 when lambda1 + lambda2 = 0; when lambda1 = lambda2 the gradient
    direction is taken as (1, 0). Returns (Oxx, Oxy, Oyy)."""
    kd = float(_get(tuning, "k_detail"))
    kn = float(_get(tuning, "k_denoise"))
    dth = float(_get(tuning, "d_th"))
    dtr = float(_get(tuning, "d_tr"))
    kst = float(_get(tuning, "k_stretch"))
    ksh = float(_get(tuning, "k_shrink"))

    t = np.stack([np.stack([ixx, ixy], -1), np.stack([ixy, iyy], -1)], -2)
    evals, evecs = np.linalg.eigh(t)            # ascending
    lam2 = evals[..., 0]
    lam1 = evals[..., 1]
    e1 = evecs[..., :, 1].copy()                # dominant eigenvector: gradient direction
    iso = (ixy == 0) & (ixx == iyy)
    e1[iso] = np.array([1.0, 0.0])

    tr = lam1 + lam2
    with np.errstate(divide="ignore", invalid="ignore"):
        A = np.where(tr > 0, 1.0 + np.sqrt((lam1 - lam2) / np.where(tr > 0, tr, 1.0)), 1.0)
    D = np.clip(1.0 - np.sqrt(lam1) / dtr + dth, 0.0, 1.0)
    k1_hat = kd * (kst * A)
    k2_hat = kd / (ksh * A)
    k1 = ((1.0 - D) * k1_hat + D * kd * kn) ** 2
    k2 = ((1.0 - D) * k2_hat + D * kd * kn) ** 2

    gx, gy = e1[..., 0], e1[..., 1]          # gradient direction
    ex, ey = -gy, gx                         # edge direction
    oxx = k1 * ex * ex + k2 * gx * gx
    oxy = k1 * ex * ey + k2 * gx * gy
    oyy = k1 * ey * ey + k2 * gy * gy
    if return_parts:
        return (oxx, oxy, oyy), dict(lam1=lam1, lam2=lam2, A=A, D=D, k1=k1, k2=k2, e1=e1)
    return oxx, oxy, oyy


# --------------------------------------------------------------------------- #
# step 5: guide statistics                                                    #
# --------------------------------------------------------------------------- #
def box3_mean_std(g):
    """3x3 colour mean and population standard deviation (edge-clamped) of a
    guide image g: [..., 3, h, w] (Sec. 5.2.2)."""
    pad = [(0, 0)] * (g.ndim - 2) + [(1, 1), (1, 1)]
    gp = np.pad(g, pad, mode="edge")
    h, w = g.shape[-2:]
    wins = [gp[..., i:i + h, j:j + w] for i in range(3) for j in range(3)]
    mean = sum(wins) / 9.0
    var = sum((wv - mean) ** 2 for wv in wins) / 9.0
    return mean, np.sqrt(var)


# --------------------------------------------------------------------------- #
# supplement S.3: high-frequency variance loss                                #
# --------------------------------------------------------------------------- #
def variance_loss(frame_ref, cfa, hf_ratio):
    """S.3: where the base frame's guide loses most of its local variance to
    the local low-pass, True. With x the guide doubled to integers (2R, G1+G2,
    2B per 2x2 quad) and S its 3x3 box sums (the low-pass, times 9), per
    channel B = 9 sum x^2 - (sum x)^2 over the 3x3 window (81 x the variance
    before) and A = 9 sum S^2 - (sum S)^2 over the 3x3 window of box sums
    (81^2 x the variance after); windows edge-replicated on the half-res grid.
    Loss where sum_c A < hf_ratio * (81 * sum_c B), exact integers compared in
    float64. hf_ratio = 0 disables the test."""
    f = np.asarray(frame_ref, dtype=np.int64)
    h, w = f.shape[0] // 2, f.shape[1] // 2
    if not hf_ratio > 0.0:
        return np.zeros((h, w), dtype=bool)
    cols = {0: (0, 1, 1, 2), 1: (1, 0, 2, 1), 2: (1, 2, 0, 1), 3: (2, 1, 1, 0)}[int(cfa)]
    quads = [f[0::2, 0::2], f[0::2, 1::2], f[1::2, 0::2], f[1::2, 1::2]]
    x = np.zeros((3, h, w), dtype=np.int64)
    for pos, c in enumerate(cols):
        x[c] += quads[pos] * (2 if c != 1 else 1)

    def win3(m):
        mp = np.pad(m, ((0, 0), (1, 1), (1, 1)), mode="edge")
        return [mp[:, i:i + h, j:j + w] for i in range(3) for j in range(3)]

    wx = win3(x)
    s_box = sum(wx)                                           # [3][h][w] 3x3 sums
    b_var = (9 * sum(v * v for v in wx) - s_box * s_box).sum(0)
    ws = win3(s_box)
    a_var = (9 * sum(v * v for v in ws) - sum(ws) ** 2).sum(0)
    return a_var.astype(np.float64) < float(hf_ratio) * (81 * b_var).astype(np.float64)


# --------------------------------------------------------------------------- #
# helpers                                                                     #
# --------------------------------------------------------------------------- #
def bilinear(m, hx, hy):
    """Bilinear sample of map m [..., h, w] at continuous indices (hx, hy)
    (x = column, y = row), with indices clamped to the map (clamp to edge).
    Leading dims of m broadcast against the sample arrays' trailing dims."""
    h, w = m.shape[-2:]
    x0 = np.floor(hx)
    y0 = np.floor(hy)
    fx = hx - x0
    fy = hy - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    xa = np.clip(x0, 0, w - 1)
    xb = np.clip(x0 + 1, 0, w - 1)
    ya = np.clip(y0, 0, h - 1)
    yb = np.clip(y0 + 1, 0, h - 1)
    top = (1.0 - fx) * m[..., ya, xa] + fx * m[..., ya, xb]
    bot = (1.0 - fx) * m[..., yb, xa] + fx * m[..., yb, xb]
    return (1.0 - fy) * top + fy * bot


def tile_grid(height, width, tile):
    return -(-height // tile), -(-width // tile)


# --------------------------------------------------------------------------- #
# step 6: motion prior                                                        #
# --------------------------------------------------------------------------- #
def motion_prior(motion_n, s1, s2, m_th):
    """Rejection strength s per tile for one frame, eqs. (7)-(8).

    M_x (M_y) is the max minus the min of the horizontal (vertical) tile
    displacements over the 3x3 tile neighbourhood (tiles outside the grid are
    skipped); M = sqrt(M_x^2 + M_y^2); s = s1 where M > M_th, else s2. The
    comparison is done as M_x^2 + M_y^2 > M_th^2 in float64 (equivalent for
    non-negative values). motion_n: [TY][TX][2]."""
    v = np.asarray(motion_n, dtype=np.float64)
    ty, tx = v.shape[:2]
    big = np.inf
    vmax = np.full((ty + 2, tx + 2, 2), -big)
    vmin = np.full((ty + 2, tx + 2, 2), big)
    vmax[1:-1, 1:-1] = v
    vmin[1:-1, 1:-1] = v
    hi = np.max(np.stack([vmax[i:i + ty, j:j + tx] for i in range(3) for j in range(3)]), axis=0)
    lo = np.min(np.stack([vmin[i:i + ty, j:j + tx] for i in range(3) for j in range(3)]), axis=0)
    mx = hi[..., 0] - lo[..., 0]
    my = hi[..., 1] - lo[..., 1]
    m_sq = mx * mx + my * my
    return np.where(m_sq > float(m_th) * float(m_th), float(s1), float(s2)), np.sqrt(m_sq)


# --------------------------------------------------------------------------- #
# step 7: robustness                                                          #
# --------------------------------------------------------------------------- #
def noise_terms(mu_ref, noise_a, noise_b, table=None):
    """Modelled guide variance sigma_md^2 and squared difference of two 3x3
    means d_md^2 per channel at the base brightness mu_ref [3][h][w] (Sec.
    5.2.2): from a Monte-Carlo table [bins][4] (R/B columns 0-1, green 2-3;
    ``oracle.noise``) when given, else the unclipped closed forms
    var = a max(mu, 0) + b (halved for the two-green mean), d_md^2 = 2 var / 9."""
    if table is not None:
        from oracle import noise as on
        t = np.asarray(table, dtype=np.float64)
        sig2 = np.stack([on.table_lookup(t, mu_ref[c], 2 if c == 1 else 0) for c in range(3)])
        dmd2 = np.stack([on.table_lookup(t, mu_ref[c], 3 if c == 1 else 1) for c in range(3)])
        return sig2, dmd2
    var = float(noise_a) * np.maximum(mu_ref, 0.0) + float(noise_b)
    var[1] = var[1] / 2.0                      # guide green = mean of two greens
    return var, 2.0 * var / 9.0


def desc_table(desc):
    """The descriptor's noise table as a numpy array, or None."""
    t = _opt(desc, "noise_table", None)
    if t is None:
        return None
    if hasattr(t, "detach"):
        t = t.detach().cpu().numpy()
    return np.asarray(t, dtype=np.float64)


def robustness(mu_ref, sd_ref, mu_n, motion_n, s_tile, t, noise_a, noise_b, tile, reject=None, table=None):
    """Robustness R on the base frame's half-resolution grid for one aligned
    frame, eqs. (5)-(6). Returns (R, R_hat) with R_hat the 5x5 minimum, eq. (9).

    Readings: the spatial sigma is the base frame's 3x3 guide sigma; the
    aligned frame's 3x3 colour mean is sampled bilinearly at u + v/2 (v = the
    displacement of the tile holding u, in full-resolution pixels); the noise
    model var(x) = a x + b (halved for the two-green mean) gives the expected
    per-pixel guide sigma sigma_md = sqrt(var) and the expected difference of
    two 3x3 means d_md = sqrt(2 var / 9), evaluated at the base mean; the three
    colour channels combine as r = sum_c d_c^2 / sum_c sigma_c^2; R is clamped
    to [0, 1]; the 5x5 minimum uses existing pixels only. ``reject`` (bool
    [h][w], optional) forces R to 0 (the full rejection of S.3)."""
    h, w = mu_ref.shape[-2:]
    ii, jj = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    ty = np.minimum((2 * ii) // tile, s_tile.shape[0] - 1)
    tx = np.minimum((2 * jj) // tile, s_tile.shape[1] - 1)
    v = np.asarray(motion_n, dtype=np.float64)[ty, tx]           # [h][w][2]
    mu_w = bilinear(mu_n, jj + v[..., 0] / 2.0, ii + v[..., 1] / 2.0)   # [3][h][w]

    var, d_md_sq = noise_terms(mu_ref, noise_a, noise_b, table)
    sigma_md = np.sqrt(var)
    sigma = np.maximum(sd_ref, sigma_md)                           # eq. (6), first line
    d_ms = mu_ref - mu_w
    d = d_ms * (d_ms * d_ms) / (d_ms * d_ms + d_md_sq)             # eq. (6), second line
    r = (d * d).sum(0) / (sigma * sigma).sum(0)
    s = s_tile[ty, tx]
    R = np.clip(s * np.exp(-r) - float(t), 0.0, 1.0)              # eq. (5)
    if reject is not None:
        R = np.where(reject, 0.0, R)
    Rp = np.pad(R, 2, mode="edge")
    R_hat = np.min(np.stack([Rp[i:i + h, j:j + w] for i in range(5) for j in range(5)]), axis=0)
    return R, R_hat


# --------------------------------------------------------------------------- #
# the merge                                                                   #
# --------------------------------------------------------------------------- #
def prepare(frames, motion, desc, tuning):
    """Steps 1-7: every per-frame map the accumulation needs."""
    frames = np.asarray(frames)
    n, h, w = frames.shape
    ref = int(_get(desc, "ref_frame"))
    cfa = int(_get(desc, "cfa"))
    tile = int(_get(desc, "tile_size"))
    x = normalise(frames, _get(desc, "black_level"), _get(desc, "white_level"))
    lum = halfres_luma(x)
    guide = halfres_guide(x, cfa)
    ixx, ixy, iyy = structure_tensor(lum)
    omega = np.stack(kernel_covariance(ixx, ixy, iyy, tuning), axis=1)   # [N][3][h][w]
    mu, sd = box3_mean_std(guide)                                         # [N][3][h][w]
    motion = np.array(motion, dtype=np.float64)
    motion[ref] = 0.0
    ty_n, tx_n = tile_grid(h, w, tile)
    assert motion.shape == (n, ty_n, tx_n, 2), motion.shape
    r_hat = np.ones((n, h // 2, w // 2))
    r_raw = np.ones((n, h // 2, w // 2))
    s_tiles = np.zeros((n, ty_n, tx_n))
    m_tiles = np.zeros((n, ty_n, tx_n))
    hf_loss = variance_loss(frames[ref], cfa, float(_opt(tuning, "hf_ratio", 0.0)))
    hf_reject = np.zeros((n, h // 2, w // 2), dtype=bool)
    for k in range(n):
        if k == ref:
            continue
        s_tiles[k], m_tiles[k] = motion_prior(motion[k], _get(tuning, "s_motion"),
                                              _get(tuning, "s"), _get(tuning, "m_th"))
        if hf_loss.any():
            # S.3: variance loss where the vector field varies strongly (the
            # motion prior's own decision, eq. 8) is fully rejected
            moving, _ = motion_prior(motion[k], 1.0, 0.0, _get(tuning, "m_th"))
            ii, jj = np.meshgrid(np.arange(h // 2), np.arange(w // 2), indexing="ij")
            ty = np.minimum((2 * ii) // tile, ty_n - 1)
            tx = np.minimum((2 * jj) // tile, tx_n - 1)
            hf_reject[k] = hf_loss & (moving[ty, tx] > 0.5)
        r_raw[k], r_hat[k] = robustness(mu[ref], sd[ref], mu[k], motion[k], s_tiles[k],
                                        _get(tuning, "t"), _get(desc, "noise_a"),
                                        _get(desc, "noise_b"), tile, hf_reject[k], desc_table(desc))
    return dict(x=x, lum=lum, guide=guide, omega=omega, mu=mu, sd=sd, motion=motion,
                r=r_raw, r_hat=r_hat, s_tiles=s_tiles, m_tiles=m_tiles, hf_reject=hf_reject,
                colours=colour_map(h, w, cfa), ref=ref, tile=tile)


def output_coords(out_h, out_w, scale):
    """Base-frame edge coordinates of the output pixel centres: ((C + 1/2) / s, (R + 1/2) / s)."""
    X = (np.arange(out_w, dtype=np.float64) + 0.5) / float(scale)
    Y = (np.arange(out_h, dtype=np.float64) + 0.5) / float(scale)
    return X, Y


def accumulate_terms(maps, X, Y):
    """Step 8 for output pixels at coordinates (X[j], Y[i]): every (value,
    exponent, robustness, colour, valid) term of eq. (1), nine per frame.

    For frame n the output pixel's position p = (X, Y) + v (v = its tile's
    displacement, 0 for the base frame) selects the 3x3 window of Bayer pixels
    around (floor p_y, floor p_x), i.e. the nine nearest samples (Sec. 5.1);
    Omega_n is sampled bilinearly at p / 2 - 1/2; the robustness of frame n is
    R_hat_n sampled bilinearly on the base grid at (X, Y) / 2 - 1/2 (1 for the
    base frame); samples outside the frame are skipped. The exponent is
    -1/2 d^T Omega^-1 d with d the sample-centre offset from p, eq. (2)."""
    x, omega, r_hat, motion = maps["x"], maps["omega"], maps["r_hat"], maps["motion"]
    n, h, w = x.shape
    tile, ref = maps["tile"], maps["ref"]
    ty_n, tx_n = motion.shape[1:3]
    Xg, Yg = np.meshgrid(X, Y)                          # [oh][ow]
    ty = np.minimum(np.floor(Yg).astype(np.int64) // tile, ty_n - 1)
    tx = np.minimum(np.floor(Xg).astype(np.int64) // tile, tx_n - 1)
    vals, exps, rhos, cols, valid = [], [], [], [], []
    for k in range(n):
        v = motion[k][ty, tx]
        px = Xg + v[..., 0]
        py = Yg + v[..., 1]
        jc = np.floor(px).astype(np.int64)
        ic = np.floor(py).astype(np.int64)
        om = bilinear(omega[k], px / 2.0 - 0.5, py / 2.0 - 0.5)     # [3][oh][ow]
        det = om[0] * om[2] - om[1] * om[1]
        ia, ib, ic_ = om[2] / det, -om[1] / det, om[0] / det        # Omega^-1
        rho = np.ones_like(Xg) if k == ref else bilinear(r_hat[k], Xg / 2.0 - 0.5, Yg / 2.0 - 0.5)
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                qi = ic + di
                qj = jc + dj
                ok = (qi >= 0) & (qi < h) & (qj >= 0) & (qj < w)
                qic = np.clip(qi, 0, h - 1)
                qjc = np.clip(qj, 0, w - 1)
                dx = (qj + 0.5) - px
                dy = (qi + 0.5) - py
                quad = ia * dx * dx + 2.0 * ib * dx * dy + ic_ * dy * dy
                vals.append(x[k][qic, qjc])
                exps.append(-0.5 * quad)
                rhos.append(rho)
                cols.append(maps["colours"][qic, qjc])
                valid.append(ok)
    return (np.stack(vals), np.stack(exps), np.stack(rhos), np.stack(cols), np.stack(valid))


def normalise_terms(vals, exps, rhos, cols, valid):
    """Step 9, eq. (1): C = sum(rho w c) / sum(rho w) per colour channel.
    Numerator and denominator are both scaled by exp(-m), m the largest
    exponent among the channel's contributing terms (rho > 0), which leaves
    the ratio unchanged and keeps the weights from underflowing."""
    out = []
    for ch in range(3):
        sel = valid & (cols == ch)
        contrib = sel & (rhos > 0)
        m = np.max(np.where(contrib, exps, -np.inf), axis=0)
        wgt = np.where(sel, rhos * np.exp(np.where(sel, exps - m, -np.inf)), 0.0)
        num = (wgt * vals).sum(0)
        den = wgt.sum(0)
        out.append(num / den)
    return np.stack(out)


def merge(frames, motion, desc, tuning, debug=False, row_block=128):
    """Merge a raw burst into linear RGB at the descriptor's output size.

    frames: uint16 [N][H][W]; motion: [N][TY][TX][2] displacements (vx, vy) of
    each base-frame tile in frame n (ignored for the base frame); desc and
    tuning: objects or dicts with the fields of hmfsr_desc / hmfsr_tuning.
    Returns float64 [3][OH][OW] (and the intermediate maps if ``debug``)."""
    maps = prepare(frames, motion, desc, tuning)
    X, Y = output_coords(int(_get(desc, "out_height")), int(_get(desc, "out_width")),
                         _get(desc, "scale"))
    out = np.empty((3, len(Y), len(X)))
    for r0 in range(0, len(Y), row_block):
        terms = accumulate_terms(maps, X, Y[r0:r0 + row_block])
        out[:, r0:r0 + row_block] = normalise_terms(*terms)
    if debug:
        return out, maps
    return out


def merge_window(frames, motion, desc, tuning, out_rows, out_cols):
    """Merge only the output pixels in the row/column index ranges given
    (slices or arrays) of the full image; the maps are still built on the
    whole input passed in."""
    maps = prepare(frames, motion, desc, tuning)
    X, Y = output_coords(int(_get(desc, "out_height")), int(_get(desc, "out_width")),
                         _get(desc, "scale"))
    return normalise_terms(*accumulate_terms(maps, X[out_cols], Y[out_rows]))
