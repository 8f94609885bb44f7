"""Brute-force per-pixel twin of the merge, for pinning the oracle on tiny inputs.

Written independently of ``oracle/merge.py``: scalar Python loops, a closed-form
2x2 eigensolver instead of LAPACK, Omega assembled as k1 I + (k2 - k1) e e^T
instead of from both eigenvectors, explicit clamped neighbourhood loops
instead of padded slices, and a per-pixel log-sum-exp normalisation. It
follows the same published definitions (Sec. 5 and S.1 of the paper) under
the same readings, so agreement to ~1e-12 pins the oracle's vectorised
indexing, padding, routing and reductions.
"""
import math

COLOURS = {0: (0, 1, 1, 2), 1: (1, 0, 2, 1), 2: (1, 2, 0, 1), 3: (2, 1, 1, 0)}


def _clamp(i, n):
    return 0 if i < 0 else (n - 1 if i >= n else i)


def _bilin(get, h, w, x, y):
    x0 = math.floor(x)
    y0 = math.floor(y)
    fx = x - x0
    fy = y - y0
    v00 = get(_clamp(y0, h), _clamp(x0, w))
    v01 = get(_clamp(y0, h), _clamp(x0 + 1, w))
    v10 = get(_clamp(y0 + 1, h), _clamp(x0, w))
    v11 = get(_clamp(y0 + 1, h), _clamp(x0 + 1, w))
    return (v00 * (1 - fx) * (1 - fy) + v01 * fx * (1 - fy)
            + v10 * (1 - fx) * fy + v11 * fx * fy)


def _eig2(a, b, c):
    """Closed-form eigen-decomposition of [[a, b], [b, c]]: (l1, l2, unit e1)."""
    half_tr = (a + c) / 2.0
    rad = math.sqrt(((a - c) / 2.0) ** 2 + b * b)
    l1, l2 = half_tr + rad, half_tr - rad
    if b == 0.0 and a == c:
        return l1, l2, (1.0, 0.0)
    if a >= c:
        ex, ey = l1 - c, b
    else:
        ex, ey = b, l1 - a
    nrm = math.hypot(ex, ey)
    return l1, l2, (ex / nrm, ey / nrm)


def brute_merge(frames, motion, desc, tuning):
    """frames: nested lists / array [N][H][W] of ints; motion [N][TY][TX][2].
    Returns [3][OH][OW] as nested lists of floats."""
    n_fr = len(frames)
    H, W = len(frames[0]), len(frames[0][0])
    h, w = H // 2, W // 2
    ref = desc.ref_frame
    T = desc.tile_size
    TY, TX = -(-H // T), -(-W // T)
    cols = COLOURS[desc.cfa]
    rng = desc.white_level - desc.black_level

    def xval(n, r, c):
        return (float(frames[n][r][c]) - desc.black_level) / rng

    def colour(r, c):
        return cols[(r & 1) * 2 + (c & 1)]

    def mv(n, ty, tx):
        if n == ref:
            return 0.0, 0.0
        return float(motion[n][ty][tx][0]), float(motion[n][ty][tx][1])

    # -- per-frame half-resolution maps, one pixel at a time
    luma = [[[0.0] * w for _ in range(h)] for _ in range(n_fr)]
    guide = [[[[0.0] * w for _ in range(h)] for _ in range(3)] for _ in range(n_fr)]
    for n in range(n_fr):
        for I in range(h):
            for J in range(w):
                vals = {}
                tot = 0.0
                for dr in (0, 1):
                    for dc in (0, 1):
                        v = xval(n, 2 * I + dr, 2 * J + dc)
                        tot += v
                        vals.setdefault(colour(2 * I + dr, 2 * J + dc), []).append(v)
                luma[n][I][J] = tot / 4.0
                for ch in range(3):
                    guide[n][ch][I][J] = sum(vals[ch]) / len(vals[ch])

    kd, kn = tuning.k_detail, tuning.k_denoise
    omega = [[[None] * w for _ in range(h)] for _ in range(n_fr)]
    for n in range(n_fr):
        L = luma[n]
        for I in range(h):
            for J in range(w):
                sxx = sxy = syy = 0.0
                for ci in (I - 1, I):
                    for cj in (J - 1, J):
                        l00 = L[_clamp(ci, h)][_clamp(cj, w)]
                        l01 = L[_clamp(ci, h)][_clamp(cj + 1, w)]
                        l10 = L[_clamp(ci + 1, h)][_clamp(cj, w)]
                        l11 = L[_clamp(ci + 1, h)][_clamp(cj + 1, w)]
                        gx = 0.5 * (l01 - l00 + l11 - l10)
                        gy = 0.5 * (l10 - l00 + l11 - l01)
                        sxx += gx * gx
                        sxy += gx * gy
                        syy += gy * gy
                a, b, c = sxx / 4.0, sxy / 4.0, syy / 4.0
                l1, l2, (gxu, gyu) = _eig2(a, b, c)
                A = 1.0 + math.sqrt((l1 - l2) / (l1 + l2)) if (l1 + l2) > 0 else 1.0
                D = min(1.0, max(0.0, 1.0 - math.sqrt(max(l1, 0.0)) / tuning.d_tr + tuning.d_th))
                k1 = ((1 - D) * kd * tuning.k_stretch * A + D * kd * kn) ** 2
                k2 = ((1 - D) * kd / (tuning.k_shrink * A) + D * kd * kn) ** 2
                # along the edge k1, along the gradient k2: Omega = k1 I + (k2 - k1) g g^T
                omega[n][I][J] = (k1 + (k2 - k1) * gxu * gxu, (k2 - k1) * gxu * gyu,
                                  k1 + (k2 - k1) * gyu * gyu)

    def box_stats(n, ch, I, J):
        vals = [guide[n][ch][_clamp(I + a, h)][_clamp(J + b, w)] for a in (-1, 0, 1) for b in (-1, 0, 1)]
        mu = sum(vals) / 9.0
        return mu, math.sqrt(sum((v - mu) ** 2 for v in vals) / 9.0)

    mu = [[[[box_stats(n, ch, I, J)[0] for J in range(w)] for I in range(h)] for ch in range(3)]
          for n in range(n_fr)]

    # -- supplement S.3: variance loss of the base frame's guide, doubled to
    # integers (Python ints: exact), 3x3 windows edge-clamped
    hf = float(getattr(tuning, "hf_ratio", 0.0))
    loss = [[False] * w for _ in range(h)]
    if hf > 0.0:
        def g2(ch, I, J):
            v = 0
            for dr in (0, 1):
                for dc in (0, 1):
                    if colour(2 * I + dr, 2 * J + dc) == ch:
                        v += int(frames[ref][2 * I + dr][2 * J + dc]) * (1 if ch == 1 else 2)
            return v

        def win(get, I, J):
            return [get(_clamp(I + a, h), _clamp(J + b, w)) for a in (-1, 0, 1) for b in (-1, 0, 1)]

        box = [[[sum(win(lambda i, j: g2(ch, i, j), I, J)) for J in range(w)] for I in range(h)]
               for ch in range(3)]
        for I in range(h):
            for J in range(w):
                A = B = 0
                for ch in range(3):
                    xs = win(lambda i, j: g2(ch, i, j), I, J)
                    ss = win(lambda i, j: box[ch][i][j], I, J)
                    B += 9 * sum(x * x for x in xs) - sum(xs) ** 2
                    A += 9 * sum(x * x for x in ss) - sum(ss) ** 2
                loss[I][J] = float(A) < hf * float(81 * B)

    # -- motion prior per (frame, tile)
    s_tile = [[[0.0] * TX for _ in range(TY)] for _ in range(n_fr)]
    moving = [[[False] * TX for _ in range(TY)] for _ in range(n_fr)]
    for n in range(n_fr):
        for ty in range(TY):
            for tx in range(TX):
                xs, ys = [], []
                for a in (-1, 0, 1):
                    for b in (-1, 0, 1):
                        if 0 <= ty + a < TY and 0 <= tx + b < TX:
                            vx, vy = mv(n, ty + a, tx + b)
                            xs.append(vx)
                            ys.append(vy)
                mx, my = max(xs) - min(xs), max(ys) - min(ys)
                moving[n][ty][tx] = mx * mx + my * my > tuning.m_th ** 2
                s_tile[n][ty][tx] = tuning.s_motion if moving[n][ty][tx] else tuning.s

    # -- robustness and its 5x5 minimum on the base grid
    R = [[[1.0] * w for _ in range(h)] for _ in range(n_fr)]
    for n in range(n_fr):
        if n == ref:
            continue
        for I in range(h):
            for J in range(w):
                ty, tx = min(2 * I // T, TY - 1), min(2 * J // T, TX - 1)
                vx, vy = mv(n, ty, tx)
                num = den = 0.0
                for ch in range(3):
                    m_ref, s_ref = box_stats(ref, ch, I, J)
                    m_al = _bilin(lambda i, j: mu[n][ch][i][j], h, w, J + vx / 2.0, I + vy / 2.0)
                    var = desc.noise_a * max(m_ref, 0.0) + desc.noise_b
                    if ch == 1:
                        var /= 2.0
                    sig = max(s_ref, math.sqrt(var))
                    dms = m_ref - m_al
                    d = dms ** 3 / (dms ** 2 + 2.0 * var / 9.0)
                    num += d * d
                    den += sig * sig
                R[n][I][J] = min(1.0, max(0.0, s_tile[n][ty][tx] * math.exp(-num / den) - tuning.t))
                if loss[I][J] and moving[n][ty][tx]:
                    R[n][I][J] = 0.0
    Rh = [[[min(R[n][_clamp(I + a, h)][_clamp(J + b, w)] for a in range(-2, 3) for b in range(-2, 3))
            for J in range(w)] for I in range(h)] for n in range(n_fr)]

    # -- accumulation per output pixel
    OH, OW, s = desc.out_height, desc.out_width, desc.scale
    out = [[[0.0] * OW for _ in range(OH)] for _ in range(3)]
    for ro in range(OH):
        Y = (ro + 0.5) / s
        for co in range(OW):
            X = (co + 0.5) / s
            ty = min(int(math.floor(Y)) // T, TY - 1)
            tx = min(int(math.floor(X)) // T, TX - 1)
            terms = [[], [], []]
            for n in range(n_fr):
                vx, vy = mv(n, ty, tx)
                px, py = X + vx, Y + vy
                oxx = _bilin(lambda i, j: omega[n][i][j][0], h, w, px / 2 - 0.5, py / 2 - 0.5)
                oxy = _bilin(lambda i, j: omega[n][i][j][1], h, w, px / 2 - 0.5, py / 2 - 0.5)
                oyy = _bilin(lambda i, j: omega[n][i][j][2], h, w, px / 2 - 0.5, py / 2 - 0.5)
                det = oxx * oyy - oxy * oxy
                rho = 1.0 if n == ref else _bilin(lambda i, j: Rh[n][i][j], h, w, X / 2 - 0.5, Y / 2 - 0.5)
                ic, jc = math.floor(py), math.floor(px)
                for qi in range(ic - 1, ic + 2):
                    for qj in range(jc - 1, jc + 2):
                        if not (0 <= qi < H and 0 <= qj < W):
                            continue
                        dx, dy = qj + 0.5 - px, qi + 0.5 - py
                        quad = (oyy * dx * dx - 2 * oxy * dx * dy + oxx * dy * dy) / det
                        terms[colour(qi, qj)].append((-0.5 * quad, rho, xval(n, qi, qj)))
            for ch in range(3):
                m = max(e for e, r, _ in terms[ch] if r > 0)
                num = sum(r * math.exp(e - m) * v for e, r, v in terms[ch])
                den = sum(r * math.exp(e - m) for e, r, v in terms[ch])
                out[ch][ro][co] = num / den
    return out
