"""Gradient of the FP64 oracle merge: finite differences and the chain rule.

TEST INFRASTRUCTURE ONLY, like ``oracle/merge.py``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU baseline leg of ``bench.py`` may use it.

The paper defines no gradient. The gradient of a loss with respect to the
tuning scalars and the per-tile displacements is, by definition, the
derivative of the oracle's forward merge (``oracle.merge.merge``). For a loss
L(C) the backward pass only sees dL/dC, so everything here is stated for the
linear functional L = sum(grad_out * C) with a given grad_out [3][OH][OW].

* ``central_difference`` / ``fd_tuning`` / ``fd_motion`` evaluate that
  definition directly: central differences of the float64 forward, accepted
  only when every discrete decision of the merge (``discrete_state``) is the
  same at theta - h, theta and theta + h, so that no kink lies in between.
* ``merge_backward`` is the chain rule of the same steps, written out in
  reverse order (eq. 1 -> eq. 2 -> eq. 4 / S.1 for the kernel covariance;
  eq. 9 -> eq. 5 -> eq. 6 for the robustness). It is checked against the
  finite differences and serves as the element-wise reference of the
  device adjoint.

Piecewise-constant decisions -- the nine-sample window centres, the cells of
every bilinear interpolation, the motion-prior choice of eq. (8), the clamps of
D (S.1) and of R (eq. 5), the 5x5 argmin of eq. (9) -- have zero derivative.
Their boundaries are kinks where the gradient is one-sided; the fingerprint
keeps finite differences away from them.

Gradient order: k_detail, k_denoise, d_th, d_tr, k_stretch, k_shrink, s, t,
s_motion (``GRAD_NAMES``).
"""
from __future__ import annotations

import hashlib

import numpy as np

from . import merge as om

GRAD_NAMES = ("k_detail", "k_denoise", "d_th", "d_tr", "k_stretch", "k_shrink", "s", "t", "s_motion")
TUNING_FIELDS = GRAD_NAMES + ("m_th",)


def tuning_dict(tuning) -> dict:
    """The tuning as a dict of float64 values (finite differences perturb it
    without the float32 rounding of the ABI structs)."""
    d = {f: float(om._get(tuning, f)) for f in TUNING_FIELDS}
    d["hf_ratio"] = float(om._opt(tuning, "hf_ratio", 0.0))
    return d


# --------------------------------------------------------------------------- #
# bilinear interpolation: derivative and transpose                            #
# --------------------------------------------------------------------------- #
def bilinear_grad(m, hx, hy):
    """``oracle.merge.bilinear`` together with its derivatives along hx and hy
    and the corner indices and weights. With the indices clamped separately,
    a clamped pair of corners coincides and the derivative across it is 0."""
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
    m_aa, m_ab = m[..., ya, xa], m[..., ya, xb]
    m_ba, m_bb = m[..., yb, xa], m[..., yb, xb]
    top = (1.0 - fx) * m_aa + fx * m_ab
    bot = (1.0 - fx) * m_ba + fx * m_bb
    val = (1.0 - fy) * top + fy * bot
    d_hx = (1.0 - fy) * (m_ab - m_aa) + fy * (m_bb - m_ba)
    d_hy = bot - top
    return val, d_hx, d_hy, (ya, yb, xa, xb, fx, fy)


def scatter_bilinear(target, cells, g):
    """Transpose of a bilinear sample: add g [...] into target [h][w] at the
    four corners with the interpolation weights."""
    ya, yb, xa, xb, fx, fy = cells
    np.add.at(target, (ya, xa), (1.0 - fx) * (1.0 - fy) * g)
    np.add.at(target, (ya, xb), fx * (1.0 - fy) * g)
    np.add.at(target, (yb, xa), (1.0 - fx) * fy * g)
    np.add.at(target, (yb, xb), fx * fy * g)


# --------------------------------------------------------------------------- #
# forward quantities the backward needs                                       #
# --------------------------------------------------------------------------- #
def _pixel_tiles(maps, Xg, Yg):
    ty_n, tx_n = maps["motion"].shape[1:3]
    tile = maps["tile"]
    ty = np.minimum(np.floor(Yg).astype(np.int64) // tile, ty_n - 1)
    tx = np.minimum(np.floor(Xg).astype(np.int64) // tile, tx_n - 1)
    return ty, tx


def _frame_samples(maps, k, Xg, Yg, ty, tx):
    """Step 8 of the forward for frame k, with what its derivative needs."""
    x, motion = maps["x"], maps["motion"]
    n, h, w = x.shape
    v = motion[k][ty, tx]
    px = Xg + v[..., 0]
    py = Yg + v[..., 1]
    jc = np.floor(px).astype(np.int64)
    ic = np.floor(py).astype(np.int64)
    om_, dom_x, dom_y, cells = bilinear_grad(maps["omega"][k], px / 2.0 - 0.5, py / 2.0 - 0.5)
    det = om_[0] * om_[2] - om_[1] * om_[1]
    inv = (om_[2] / det, -om_[1] / det, om_[0] / det)
    if k == maps["ref"]:
        rho = np.ones_like(Xg)
    else:
        rho = om.bilinear(maps["r_hat"][k], Xg / 2.0 - 0.5, Yg / 2.0 - 0.5)
    dxs, dys, exps, vals, cols, valid = [], [], [], [], [], []
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            qi, qj = ic + di, jc + dj
            ok = (qi >= 0) & (qi < h) & (qj >= 0) & (qj < w)
            qic, qjc = np.clip(qi, 0, h - 1), np.clip(qj, 0, w - 1)
            dx = (qj + 0.5) - px
            dy = (qi + 0.5) - py
            quad = inv[0] * dx * dx + 2.0 * inv[1] * dx * dy + inv[2] * dy * dy
            dxs.append(dx)
            dys.append(dy)
            exps.append(-0.5 * quad)
            vals.append(x[k][qic, qjc])
            cols.append(maps["colours"][qic, qjc])
            valid.append(ok)
    return dict(px=px, py=py, jc=jc, ic=ic, omega=om_, dom_x=dom_x, dom_y=dom_y, cells=cells,
                inv=inv, rho=rho, dx=np.stack(dxs), dy=np.stack(dys), e=np.stack(exps),
                val=np.stack(vals), col=np.stack(cols), valid=np.stack(valid))


def _robust_parts(maps, k, desc, tuning):
    """Steps 6-7 for aligned frame k with the unclamped R, the derivative of
    the sampled colour mean and the motion-prior decision per pixel."""
    mu, sd, motion = maps["mu"], maps["sd"], maps["motion"]
    ref, tile = maps["ref"], maps["tile"]
    h, w = mu.shape[-2:]
    ii, jj = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    ty = np.minimum((2 * ii) // tile, motion.shape[1] - 1)
    tx = np.minimum((2 * jj) // tile, motion.shape[2] - 1)
    v = motion[k][ty, tx]
    mu_w, dmu_x, dmu_y, cells = bilinear_grad(mu[k], jj + v[..., 0] / 2.0, ii + v[..., 1] / 2.0)
    mu_ref, sd_ref = mu[ref], sd[ref]
    var, d_md_sq = om.noise_terms(mu_ref, om._get(desc, "noise_a"), om._get(desc, "noise_b"),
                                  om.desc_table(desc))
    sigma = np.maximum(sd_ref, np.sqrt(var))
    d_ms = mu_ref - mu_w
    d = d_ms * (d_ms * d_ms) / (d_ms * d_ms + d_md_sq)
    sig2 = (sigma * sigma).sum(0)
    r = (d * d).sum(0) / sig2
    # which rejection strength each tile uses: the eq. (8) decision itself
    moving, _ = om.motion_prior(motion[k], 1.0, 0.0, om._get(tuning, "m_th"))
    moving = moving[ty, tx] > 0.5
    s = np.where(moving, float(om._get(tuning, "s_motion")), float(om._get(tuning, "s")))
    r_raw = s * np.exp(-r) - float(om._get(tuning, "t"))
    # S.3 full rejection: R held at 0 there, like a clamp
    r_raw = np.where(maps["hf_reject"][k], -1.0, r_raw)
    return dict(ty=ty, tx=tx, dmu_x=dmu_x, dmu_y=dmu_y, cells=cells, d_ms=d_ms, d_md_sq=d_md_sq,
                d=d, sig2=sig2, r=r, s=s, moving=moving, r_raw=r_raw)


def _argmin5(R):
    """Index of the 5x5 minimum of eq. (9) per pixel: edge-replicated window
    scanned row by row, first minimum wins. Returns (rows, cols)."""
    h, w = R.shape
    ii, jj = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    cand_i, cand_j = [], []
    for di in range(-2, 3):
        for dj in range(-2, 3):
            cand_i.append(np.clip(ii + di, 0, h - 1))
            cand_j.append(np.clip(jj + dj, 0, w - 1))
    cand_i, cand_j = np.stack(cand_i), np.stack(cand_j)
    best = np.argmin(R[cand_i, cand_j], axis=0)
    return (np.take_along_axis(cand_i, best[None], 0)[0], np.take_along_axis(cand_j, best[None], 0)[0])


def _omega_parts(maps, k, tuning):
    ixx, ixy, iyy = om.structure_tensor(maps["lum"][k])
    _, parts = om.kernel_covariance(ixx, ixy, iyy, tuning, return_parts=True)
    d_raw = 1.0 - np.sqrt(parts["lam1"]) / float(om._get(tuning, "d_tr")) + float(om._get(tuning, "d_th"))
    parts["d_raw"] = d_raw
    return parts


# --------------------------------------------------------------------------- #
# discrete state                                                              #
# --------------------------------------------------------------------------- #
def discrete_state(frames, motion, desc, tuning) -> str:
    """Digest of every piecewise-constant decision of the forward merge."""
    maps = om.prepare(frames, motion, desc, tuning)
    X, Y = om.output_coords(int(om._get(desc, "out_height")), int(om._get(desc, "out_width")),
                            om._get(desc, "scale"))
    Xg, Yg = np.meshgrid(X, Y)
    ty, tx = _pixel_tiles(maps, Xg, Yg)
    hsh = hashlib.sha1()
    n = maps["x"].shape[0]
    for k in range(n):
        v = maps["motion"][k][ty, tx]
        px, py = Xg + v[..., 0], Yg + v[..., 1]
        for a in (np.floor(px), np.floor(py), np.floor(px / 2.0 - 0.5), np.floor(py / 2.0 - 0.5)):
            hsh.update(a.astype(np.int64).tobytes())
        parts = _omega_parts(maps, k, tuning)
        hsh.update(np.digitize(parts["d_raw"], [0.0, 1.0], right=False).astype(np.int8).tobytes())
        hsh.update((parts["d_raw"] == 0.0).tobytes() + (parts["d_raw"] == 1.0).tobytes())
        if k == maps["ref"]:
            continue
        rp = _robust_parts(maps, k, desc, tuning)
        hsh.update(rp["moving"].tobytes())
        hsh.update(np.digitize(rp["r_raw"], [0.0, 1.0]).astype(np.int8).tobytes())
        hsh.update((rp["r_raw"] == 0.0).tobytes() + (rp["r_raw"] == 1.0).tobytes())
        ya, yb, xa, xb, _, _ = rp["cells"]
        hsh.update(ya.tobytes() + yb.tobytes() + xa.tobytes() + xb.tobytes())
        ai, aj = _argmin5(maps["r"][k])
        hsh.update(ai.tobytes() + aj.tobytes())
        rho = om.bilinear(maps["r_hat"][k], Xg / 2.0 - 0.5, Yg / 2.0 - 0.5)
        hsh.update((rho > 0).tobytes())
    return hsh.hexdigest()


# --------------------------------------------------------------------------- #
# finite differences (the definition)                                         #
# --------------------------------------------------------------------------- #
def loss(frames, motion, desc, tuning, grad_out) -> float:
    """L = sum(grad_out * C), C the oracle merge."""
    return float(np.sum(np.asarray(grad_out, np.float64) * om.merge(frames, motion, desc, tuning)))


def central_difference(f, state, h, max_halvings=5):
    """(f(h) - f(-h)) / 2h for f(delta) = loss at theta + delta, with the step
    halved until state(-h) == state(0) == state(h). Returns (g, h) or
    (None, h) when no admissible step was found."""
    s0 = state(0.0)
    for _ in range(max_halvings + 1):
        if state(h) == s0 and state(-h) == s0:
            return (f(h) - f(-h)) / (2.0 * h), h
        h *= 0.5
    return None, h


def fd_tuning(frames, motion, desc, tuning, grad_out, name, rel_h=1e-4):
    """Central difference of L in tuning scalar ``name``, step 1e-4 * |theta|
    (relative: D_th and D_tr are ~1e-2, where a fixed 1e-4 step would be 1 %
    of the value and its truncation error alone would reach 1e-3)."""
    base = tuning_dict(tuning)
    theta = base[name]

    def at(delta):
        t = dict(base)
        t[name] = theta + delta
        return t

    return central_difference(lambda dl: loss(frames, motion, desc, at(dl), grad_out),
                              lambda dl: discrete_state(frames, motion, desc, at(dl)),
                              rel_h * (abs(theta) if theta != 0.0 else 1.0))


def fd_motion(frames, motion, desc, tuning, grad_out, k, ty, tx, comp, h=1e-4):
    """Central difference of L in motion[k][ty][tx][comp] (step 1e-4 px)."""
    base = np.array(motion, dtype=np.float64)
    tun = tuning_dict(tuning)

    def at(delta):
        m = base.copy()
        m[k, ty, tx, comp] += delta
        return m

    return central_difference(lambda dl: loss(frames, at(dl), desc, tun, grad_out),
                              lambda dl: discrete_state(frames, at(dl), desc, tun), h)


# --------------------------------------------------------------------------- #
# the chain rule                                                              #
# --------------------------------------------------------------------------- #
def _accumulate_block(maps, X, Yb, grad_out, g_omega, g_rhat, g_motion):
    """Backward of steps 8-9 for output rows Yb: dL/dOmega_n (per half-res
    pixel, all frames), dL/dR_hat_n (aligned frames) and the direct part of
    dL/dv (through the sample offsets and the Omega sampling position)."""
    n = maps["x"].shape[0]
    ref = maps["ref"]
    Xg, Yg = np.meshgrid(X, Yb)
    ty, tx = _pixel_tiles(maps, Xg, Yg)
    fr = [_frame_samples(maps, k, Xg, Yg, ty, tx) for k in range(n)]
    # eq. (1): per channel normaliser, as the forward computes it
    E = np.stack([f["e"] for f in fr])                     # [n][9][oh][ow]
    V = np.stack([f["val"] for f in fr])
    COL = np.stack([f["col"] for f in fr])
    OK = np.stack([f["valid"] for f in fr])
    RHO = np.stack([f["rho"] for f in fr])[:, None]        # [n][1][oh][ow]
    b = np.zeros_like(E)                                   # dL/drho per term
    for ch in range(3):
        contrib = OK & (COL == ch) & (RHO > 0)
        m = np.max(np.where(contrib, E, -np.inf), axis=(0, 1))
        ew = np.where(contrib, np.exp(np.where(contrib, E - m, 0.0)), 0.0)
        den = (RHO * ew).sum((0, 1))
        C = (RHO * ew * V).sum((0, 1)) / den
        # C = sum(rho w c) / sum(rho w): dC/d(rho_i) = w_i (c_i - C) / den
        b += np.where(contrib, ew * (V - C) * (grad_out[ch] / den), 0.0)
    a = RHO * b                                            # dL/de per term (dC/de_i = rho_i w_i (c_i - C) / den)
    for k in range(n):
        f = fr[k]
        ia, ib, ic = f["inv"]
        # e = -1/2 d^T Omega^-1 d with d = q + 1/2 - p:  de/dp = u = Omega^-1 d,
        # de/dOmega = 1/2 u u^T (Oxy counted on both off-diagonal entries).
        ux = ia * f["dx"] + ib * f["dy"]
        uy = ib * f["dx"] + ic * f["dy"]
        ak = a[k]
        g_px = (ak * ux).sum(0)
        g_py = (ak * uy).sum(0)
        g_om = np.stack([(0.5 * ak * ux * ux).sum(0), (ak * ux * uy).sum(0), (0.5 * ak * uy * uy).sum(0)])
        # Omega is sampled at p / 2 - 1/2
        g_px += 0.5 * (g_om * f["dom_x"]).sum(0)
        g_py += 0.5 * (g_om * f["dom_y"]).sum(0)
        for c in range(3):
            scatter_bilinear(g_omega[k][c], f["cells"], g_om[c])
        if k == ref:
            continue
        np.add.at(g_motion[k][..., 0], (ty, tx), g_px)
        np.add.at(g_motion[k][..., 1], (ty, tx), g_py)
        g_rho = b[k].sum(0)
        _, _, _, rcells = bilinear_grad(maps["r_hat"][k], Xg / 2.0 - 0.5, Yg / 2.0 - 0.5)
        scatter_bilinear(g_rhat[k], rcells, g_rho)


def omega_backward(maps, g_omega, tuning):
    """dL/d(k_detail, k_denoise, d_th, d_tr, k_stretch, k_shrink) from
    dL/dOmega_n of every frame, through eq. (4) and the S.1 heuristics."""
    kd = float(om._get(tuning, "k_detail"))
    kn = float(om._get(tuning, "k_denoise"))
    dtr = float(om._get(tuning, "d_tr"))
    kst = float(om._get(tuning, "k_stretch"))
    ksh = float(om._get(tuning, "k_shrink"))
    g = np.zeros(6)
    for k in range(g_omega.shape[0]):
        p = _omega_parts(maps, k, tuning)
        gxx, gxy, gyy = g_omega[k]
        ex_g, ey_g = p["e1"][..., 0], p["e1"][..., 1]      # gradient direction
        ex_e, ey_e = -ey_g, ex_g                           # edge direction
        # Omega = k1 e_edge e_edge^T + k2 e_grad e_grad^T
        g_k1 = gxx * ex_e * ex_e + gxy * ex_e * ey_e + gyy * ey_e * ey_e
        g_k2 = gxx * ex_g * ex_g + gxy * ex_g * ey_g + gyy * ey_g * ey_g
        A, D = p["A"], p["D"]
        k1_hat = kd * kst * A
        k2_hat = kd / (ksh * A)
        sig1 = (1.0 - D) * k1_hat + D * kd * kn             # k1 = sig1^2
        sig2 = (1.0 - D) * k2_hat + D * kd * kn
        g_s1 = 2.0 * sig1 * g_k1
        g_s2 = 2.0 * sig2 * g_k2
        g[0] += np.sum(g_s1 * ((1.0 - D) * kst * A + D * kn) + g_s2 * ((1.0 - D) / (ksh * A) + D * kn))
        g[1] += np.sum((g_s1 + g_s2) * D * kd)
        g_D = g_s1 * (kd * kn - k1_hat) + g_s2 * (kd * kn - k2_hat)
        inside = (p["d_raw"] > 0.0) & (p["d_raw"] < 1.0)   # D = clamp(1 - sqrt(l1)/D_tr + D_th)
        g[2] += np.sum(np.where(inside, g_D, 0.0))
        g[3] += np.sum(np.where(inside, g_D * np.sqrt(p["lam1"]) / (dtr * dtr), 0.0))
        g[4] += np.sum(g_s1 * (1.0 - D) * kd * A)
        g[5] += np.sum(g_s2 * (1.0 - D) * kd * (-1.0 / (ksh * ksh * A)))
    return g


def robustness_backward(maps, g_rhat, desc, tuning, g_motion):
    """dL/d(s, t, s_motion) and the robustness part of dL/dv from dL/dR_hat_n,
    through the 5x5 minimum (eq. 9), the clamp and exponential of eq. (5) and
    the noise-corrected distance of eq. (6). Adds into g_motion."""
    g = np.zeros(3)      # s, t, s_motion
    for k in range(g_rhat.shape[0]):
        if k == maps["ref"]:
            continue
        ai, aj = _argmin5(maps["r"][k])
        g_R = np.zeros_like(g_rhat[k])
        np.add.at(g_R, (ai, aj), g_rhat[k])
        rp = _robust_parts(maps, k, desc, tuning)
        inside = (rp["r_raw"] > 0.0) & (rp["r_raw"] < 1.0)
        g_R = np.where(inside, g_R, 0.0)
        ex = np.exp(-rp["r"])
        g_sv = g_R * ex
        g[0] += np.sum(np.where(rp["moving"], 0.0, g_sv))
        g[2] += np.sum(np.where(rp["moving"], g_sv, 0.0))
        g[1] -= np.sum(g_R)
        g_r = -g_R * rp["s"] * ex
        # r = sum_c d_c^2 / sum_c sigma_c^2; d = d_ms^3 / (d_ms^2 + d_md^2); d_ms = mu_ref - mu_w
        dms2 = rp["d_ms"] ** 2
        dd_ddms = dms2 * (dms2 + 3.0 * rp["d_md_sq"]) / (dms2 + rp["d_md_sq"]) ** 2
        g_muw = -(g_r * 2.0 * rp["d"] / rp["sig2"]) * dd_ddms          # [3][h][w]
        # mu_w is sampled at u + v / 2
        g_vx = 0.5 * (g_muw * rp["dmu_x"]).sum(0)
        g_vy = 0.5 * (g_muw * rp["dmu_y"]).sum(0)
        np.add.at(g_motion[k][..., 0], (rp["ty"], rp["tx"]), g_vx)
        np.add.at(g_motion[k][..., 1], (rp["ty"], rp["tx"]), g_vy)
    return g


def merge_backward(frames, motion, desc, tuning, grad_out, row_block=64):
    """Gradient of L = sum(grad_out * merge(...)). Returns (g_tuning [9] in
    ``GRAD_NAMES`` order, g_motion [N][TY][TX][2] with the base frame's row 0)."""
    maps = om.prepare(frames, motion, desc, tuning)
    grad_out = np.asarray(grad_out, np.float64)
    n, H, W = maps["x"].shape
    X, Y = om.output_coords(int(om._get(desc, "out_height")), int(om._get(desc, "out_width")),
                            om._get(desc, "scale"))
    g_omega = np.zeros((n, 3, H // 2, W // 2))
    g_rhat = np.zeros((n, H // 2, W // 2))
    g_motion = np.zeros(maps["motion"].shape)
    for r0 in range(0, len(Y), row_block):
        _accumulate_block(maps, X, Y[r0:r0 + row_block], grad_out[:, r0:r0 + row_block],
                          g_omega, g_rhat, g_motion)
    g6 = omega_backward(maps, g_omega, tuning)
    g3 = robustness_backward(maps, g_rhat, desc, tuning, g_motion)
    g_motion[maps["ref"]] = 0.0
    return np.concatenate([g6, g3[[0, 1, 2]]]), g_motion
