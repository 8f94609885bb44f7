"""FP64 / integer CPU oracle of the tile alignment that produces the merge's
motion vectors.

TEST INFRASTRUCTURE ONLY, like ``oracle/merge.py``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU baseline leg of ``bench.py`` may use it.

The paper registers every frame against the base frame per tile (Sec. 3.2):
a coarse-to-fine pyramid block matching (the burst pipeline it builds on)
followed by three Lucas-Kanade iterations that refine the block-matching
vectors to subpixel accuracy. It gives no further detail; the readings below
fill it in and are shared with the device code.

Readings:
  * the image aligned is the half-resolution luma of 2x2 Bayer quads (as in
    Sec. 5.1.2), kept as integer quad sums (the black level cancels in every
    difference);
  * pyramid level l+1 holds the 2x2 sums of level l (size halved, odd last
    row/column dropped); levels are added while the coarser level still holds
    a whole block, up to ``levels`` in total;
  * blocks: on level 0 the merge's tiles (T_s/2 half-res pixels, so that the
    vectors land on the merge's tile grid); on coarser levels 8x8 pixels;
  * block matching on a level: candidate offsets are the guess plus every
    integer (dx, dy) with |dx|, |dy| <= R (R = ``radius_coarse`` on the
    coarsest level, ``radius_fine`` elsewhere); the cost is the sum of squared
    differences over the block's pixels inside the level image, the moved frame
    sampled with edge-replicated indices; the minimum cost wins, ties going to
    the smallest dx^2 + dy^2, then to the first in row-major scan order;
  * the guess for a block is twice the vector of the coarser level's block that
    holds the block's centre (zero on the coarsest level);
  * noise gate (kappa = ``gate`` >= 0, default 4; 0 turns it off): a block
    keeps its guess unless the winner lowers the cost by more than kappa
    standard deviations of what noise alone moves a cost difference by. With
    the noise model of Sec. 5.2.2 every raw value x (normalised to [0, 1] by
    black and white level) has variance (a x + b) R^2 in raw units, R = white -
    black; a level-l pixel sums m = 4^(l+1) raw values, so its variance is
    v = m (a x + b) R^2, x taken at the block's mean (clamped to [0, 1]). For
    two candidates over N pixels of noise only, the cost difference
    sum (n1 - n0)^2 - (n2 - n0)^2 has variance 12 N v^2. The test is taken
    without divisions or roots, in float64 with every operation rounded in
    the order written: with S the block's integer sum, e = clamp(S - N m black,
    0, N m R) and u = a R e + N m b R R (= N v), the block moves iff
    N gain^2 > 12 kappa^2 u^2, gain = SSD(guess) - SSD(winner). It stops noise
    from steering flat blocks and blocks along straight edges (the aperture
    problem) off their guess; content that moves (or aliases) gains far more
    than that and is matched as before;
  * Lucas-Kanade on level 0 (translation only, template gradients): with
    g(p) the central-difference gradient of the base image (edge-replicated)
    and e(p) = I_n(p + v) - I_0(p) (I_n sampled bilinearly, edge-clamped as in
    the merge), H = sum g g^T and b = sum g e over the tile's window,
    v <- v - H^-1 b; a tile with det H <= 1e-9 (tr H)^2 keeps its vector.
    The window is the tile grown by half a tile on every side and clipped to
    the image (overlapping windows, as the burst pipeline's tiles overlap by
    half), which halves the noise of the estimate on small tiles;
  * the result is 2 v (half-res pixels -> Bayer pixels); the base frame's
    vectors are 0.
"""
from __future__ import annotations

import numpy as np

DEFAULTS = dict(levels=4, radius_coarse=4, radius_fine=2, lk_iterations=3, coarse_block=8, gate=4.0)


def quad_sums(frame):
    """Integer 2x2 quad sums of a raw frame [H][W] -> [H/2][W/2] int64."""
    f = np.asarray(frame, dtype=np.int64)
    return f[0::2, 0::2] + f[0::2, 1::2] + f[1::2, 0::2] + f[1::2, 1::2]


def pyramid(gray, levels, block):
    """Level 0 = gray; level l+1 = 2x2 sums of level l, while it holds a block."""
    pyr = [gray]
    while len(pyr) < levels:
        g = pyr[-1]
        h, w = g.shape[0] // 2, g.shape[1] // 2
        if h < block or w < block:
            break
        g = g[:2 * h, :2 * w]
        pyr.append(g[0::2, 0::2] + g[0::2, 1::2] + g[1::2, 0::2] + g[1::2, 1::2])
    return pyr


def block_grid(shape, block):
    return -(-shape[0] // block), -(-shape[1] // block)


def noise_gate_moves(tpl, level, gain, gate, noise):
    """The noise gate's decision for a block ``tpl`` of pyramid level ``level``
    whose best candidate lowers the cost by the integer ``gain``: True when
    the move is significant. noise = (a, b, black, white) of the descriptor
    (float32 values); every float64 operation below is rounded in the order
    written, as the device code does it."""
    a, b, black, white = (float(np.float32(x)) for x in noise)
    kappa = float(np.float32(gate))
    rng = white - black
    n = float(tpl.size)
    nm = n * (4.0 ** (level + 1))
    e = float(int(np.sum(tpl, dtype=np.int64))) - nm * black
    e = min(max(e, 0.0), nm * rng)
    u = (a * rng) * e + ((nm * b) * rng) * rng
    g = float(gain)
    return (n * g) * g > (((12.0 * kappa) * kappa) * u) * u


def match_block(base, img, block, by, bx, guess, radius, gate=0.0, noise=None, level=0):
    """Integer offset (ux, uy) of block (by, bx) of ``base`` found in ``img``:
    minimum SSD over guess + [-R, R]^2, ties to the smallest dx^2 + dy^2,
    then to the first candidate in row-major order; with gate > 0 the guess
    is kept unless ``noise_gate_moves`` finds the winner's gain significant."""
    h, w = base.shape
    ys = np.arange(by * block, min(by * block + block, h))
    xs = np.arange(bx * block, min(bx * block + block, w))
    tpl = base[np.ix_(ys, xs)]
    gx, gy = int(guess[0]), int(guess[1])
    best = None
    k = 0
    for dy in range(-radius, radius + 1):
        for dx in range(-radius, radius + 1):
            ux, uy = gx + dx, gy + dy
            yy = np.clip(ys + uy, 0, h - 1)
            xx = np.clip(xs + ux, 0, w - 1)
            diff = img[np.ix_(yy, xx)] - tpl
            key = (int(np.sum(diff * diff)), dx * dx + dy * dy, k)
            if dx == 0 and dy == 0:
                ssd_guess = key[0]
            if best is None or key < best[0]:
                best = (key, ux, uy)
            k += 1
    if gate > 0 and not noise_gate_moves(tpl, level, ssd_guess - best[0][0], gate, noise):
        return gx, gy
    return best[1], best[2]


def match_level(base, img, block, guess, radius, gate=0.0, noise=None, level=0):
    """Block matching of one level. guess: [BY][BX][2] integer (dx, dy).
    Returns the chosen integer offsets [BY][BX][2]."""
    by_n, bx_n = block_grid(base.shape, block)
    out = np.zeros((by_n, bx_n, 2), dtype=np.int64)
    for by in range(by_n):
        for bx in range(bx_n):
            out[by, bx] = match_block(base, img, block, by, bx, guess[by, bx], radius, gate, noise, level)
    return out


def coarse_parent(b, block, coarse_block, n_coarse):
    """Index of the coarser-level block that holds the centre of block b."""
    return min(int(((b + 0.5) * block) / 2.0 // coarse_block), n_coarse - 1)


def upsample_guess(coarse_vec, coarse_block, shape, block):
    """Guess per block of a finer level: twice the vector of the coarser
    block holding the block's centre."""
    by_n, bx_n = block_grid(shape, block)
    cy_n, cx_n = coarse_vec.shape[:2]
    out = np.zeros((by_n, bx_n, 2), dtype=np.int64)
    for by in range(by_n):
        cy = coarse_parent(by, block, coarse_block, cy_n)
        for bx in range(bx_n):
            out[by, bx] = 2 * coarse_vec[cy, coarse_parent(bx, block, coarse_block, cx_n)]
    return out


def bilinear_clamped(img, x, y):
    """Bilinear sample with separately clamped corner indices (as the merge's)."""
    h, w = img.shape
    x0 = np.floor(x)
    y0 = np.floor(y)
    fx, fy = x - x0, y - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    xa, xb = np.clip(x0, 0, w - 1), np.clip(x0 + 1, 0, w - 1)
    ya, yb = np.clip(y0, 0, h - 1), np.clip(y0 + 1, 0, h - 1)
    top = (1.0 - fx) * img[ya, xa] + fx * img[ya, xb]
    bot = (1.0 - fx) * img[yb, xa] + fx * img[yb, xb]
    return (1.0 - fy) * top + fy * bot


def lk_window(by, bx, block, shape):
    """Rows and columns of the Lucas-Kanade window of tile (by, bx)."""
    h, w = shape
    m = block // 2
    ys = np.arange(max(0, by * block - m), min(by * block + block + m, h))
    xs = np.arange(max(0, bx * block - m), min(bx * block + block + m, w))
    return ys, xs


def central_gradient(img):
    """(d/dx, d/dy) by central differences with edge-replicated indices."""
    h, w = img.shape
    b = img.astype(np.float64)
    gx = (b[:, np.minimum(np.arange(w) + 1, w - 1)] - b[:, np.maximum(np.arange(w) - 1, 0)]) / 2.0
    gy = (b[np.minimum(np.arange(h) + 1, h - 1), :] - b[np.maximum(np.arange(h) - 1, 0), :]) / 2.0
    return gx, gy


def lk_refine(base_f, img_f, gx, gy, ys, xs, v, iterations):
    """Lucas-Kanade iterations for one window; returns the refined (vx, vy)."""
    Y, X = np.meshgrid(ys, xs, indexing="ij")
    g1, g2 = gx[Y, X], gy[Y, X]
    hxx, hxy, hyy = np.sum(g1 * g1), np.sum(g1 * g2), np.sum(g2 * g2)
    det = hxx * hyy - hxy * hxy
    tr = hxx + hyy
    vx, vy = float(v[0]), float(v[1])
    if not (tr > 0.0 and det > 1e-9 * tr * tr):
        return vx, vy
    tpl = base_f[Y, X]
    for _ in range(iterations):
        e = bilinear_clamped(img_f, X + vx, Y + vy) - tpl
        sx, sy = np.sum(g1 * e), np.sum(g2 * e)
        vx -= (hyy * sx - hxy * sy) / det
        vy -= (hxx * sy - hxy * sx) / det
    return vx, vy


def lucas_kanade(base, img, block, v0, iterations):
    """Translation-only Lucas-Kanade refinement of every tile on level 0."""
    base_f = base.astype(np.float64)
    img_f = img.astype(np.float64)
    gx, gy = central_gradient(base)
    by_n, bx_n = block_grid(base.shape, block)
    v = v0.astype(np.float64).copy()
    for by in range(by_n):
        for bx in range(bx_n):
            ys, xs = lk_window(by, bx, block, base.shape)
            v[by, bx] = lk_refine(base_f, img_f, gx, gy, ys, xs, v0[by, bx], iterations)
    return v


def align(frames, desc, params=None, debug=False):
    """Per-tile motion [N][TY][TX][2] (Bayer pixels, float64) of every frame
    against the base frame. frames: uint16 [N][H][W]."""
    p = dict(DEFAULTS)
    p.update(params or {})
    frames = np.asarray(frames)
    n = frames.shape[0]
    ref = int(desc.ref_frame if not isinstance(desc, dict) else desc["ref_frame"])
    tile = int(desc.tile_size if not isinstance(desc, dict) else desc["tile_size"])
    noise = desc_noise(desc)
    b0 = tile // 2
    grays = [quad_sums(frames[k]) for k in range(n)]
    pyr_ref, blocks = _levels_and_blocks(grays[ref], tile, p)
    nl = len(pyr_ref)
    ty_n, tx_n = block_grid(grays[ref].shape, b0)
    motion = np.zeros((n, ty_n, tx_n, 2))
    steps = {}
    for k in range(n):
        if k == ref:
            continue
        pyr = pyramid(grays[k], nl, p["coarse_block"])
        vec = None
        per_level = []
        for lv in range(nl - 1, -1, -1):
            shape = pyr_ref[lv].shape
            if vec is None:
                guess = np.zeros(block_grid(shape, blocks[lv]) + (2,), dtype=np.int64)
                radius = p["radius_coarse"]
            else:
                guess = upsample_guess(vec, blocks[lv + 1], shape, blocks[lv])
                radius = p["radius_fine"]
            vec = match_level(pyr_ref[lv], pyr[lv], blocks[lv], guess, radius, p["gate"], noise, lv)
            per_level.append(vec)
        v = lucas_kanade(pyr_ref[0], pyr[0], b0, vec, p["lk_iterations"])
        motion[k] = 2.0 * v
        steps[k] = dict(block_match=vec, levels=per_level[::-1])
    if debug:
        return motion, steps
    return motion


def desc_noise(desc):
    """(noise_a, noise_b, black_level, white_level) of a descriptor or of a
    dict (missing keys: 1e-3, 1e-6, 64, 4095, the 12-bit defaults)."""
    names = (("noise_a", 1e-3), ("noise_b", 1e-6), ("black_level", 64.0), ("white_level", 4095.0))
    if isinstance(desc, dict):
        return tuple(float(desc.get(k, v)) for k, v in names)
    return tuple(float(getattr(desc, k)) for k, _ in names)


def _levels_and_blocks(grays_ref, tile, p):
    pyr_ref = pyramid(grays_ref, p["levels"], p["coarse_block"])
    blocks = [tile // 2] + [p["coarse_block"]] * (len(pyr_ref) - 1)
    return pyr_ref, blocks


def align_sampled(frames, desc, frame, tiles, params=None):
    """Motion of a few level-0 tiles of one frame, for bursts too large for
    ``align``: only the chain of coarser blocks each tile's guess comes from is
    matched. tiles: iterable of (ty, tx). Returns (motion [len][2] float64 in
    Bayer pixels, block-matching vectors [len][2] int64 in half-res pixels)."""
    p = dict(DEFAULTS)
    p.update(params or {})
    frames = np.asarray(frames)
    ref = int(desc.ref_frame if not isinstance(desc, dict) else desc["ref_frame"])
    tile = int(desc.tile_size if not isinstance(desc, dict) else desc["tile_size"])
    noise = desc_noise(desc)
    tiles = [(int(a), int(b)) for a, b in tiles]
    if frame == ref:
        return np.zeros((len(tiles), 2)), np.zeros((len(tiles), 2), dtype=np.int64)
    pyr_ref, blocks = _levels_and_blocks(quad_sums(frames[ref]), tile, p)
    nl = len(pyr_ref)
    pyr = pyramid(quad_sums(frames[frame]), nl, p["coarse_block"])
    grids = [block_grid(pyr_ref[lv].shape, blocks[lv]) for lv in range(nl)]
    memo = {}

    def vec(lv, by, bx):
        key = (lv, by, bx)
        if key not in memo:
            if lv == nl - 1:
                guess = (0, 0)
                radius = p["radius_coarse"]
            else:
                cy = coarse_parent(by, blocks[lv], blocks[lv + 1], grids[lv + 1][0])
                cx = coarse_parent(bx, blocks[lv], blocks[lv + 1], grids[lv + 1][1])
                g = vec(lv + 1, cy, cx)
                guess = (2 * g[0], 2 * g[1])
                radius = p["radius_fine"]
            memo[key] = match_block(pyr_ref[lv], pyr[lv], blocks[lv], by, bx, guess, radius, p["gate"], noise, lv)
        return memo[key]

    base_f = pyr_ref[0].astype(np.float64)
    img_f = pyr[0].astype(np.float64)
    gx, gy = central_gradient(pyr_ref[0])
    motion = np.zeros((len(tiles), 2))
    bm = np.zeros((len(tiles), 2), dtype=np.int64)
    for i, (ty, tx) in enumerate(tiles):
        bm[i] = vec(0, ty, tx)
        ys, xs = lk_window(ty, tx, blocks[0], pyr_ref[0].shape)
        vx, vy = lk_refine(base_f, img_f, gx, gy, ys, xs, bm[i], p["lk_iterations"])
        motion[i] = (2.0 * vx, 2.0 * vy)
    return motion, bm
