// Fused output-tile merge (Sec. 5.1, eq. 1-2 with the kernel covariance of
// Sec. 5.1.2 / S.1 and the robustness of Sec. 5.2).
//
// One workgroup owns a 64x32 output tile: lane = column, wave w = rows
// 8w..8w+7, so every thread keeps the per-channel accumulators of 8 pixels in
// registers for the whole burst (the paper's online merge: memory does not
// grow with the frame count). For each frame, base frame first:
//   1. the frame's tile displacements and the tile's R_hat window are staged;
//   2. the warped footprint (nine-sample windows plus the structure-tensor
//      border) is found by a block reduction over the pixels' positions;
//   3. the raw Bayer footprint is copied to LDS, 2x2-quad sums (luma) and the
//      kernel covariance Omega (float64) are computed for the footprint;
//   4. every pixel interpolates Omega and R_hat bilinearly, forms the nine
//      exponents in float64, and accumulates exp2-weighted raw values per
//      channel against a per-channel reference exponent that is raised only
//      when a frame would exceed it by more than 2^64 (online normalisation).
// If a frame's footprint does not fit the LDS buffers (a strongly divergent
// motion field), the tile is processed one alignment tile at a time.
#include <math.h>

#include "hmfsr_internal.h"
#include "omega.h"

namespace hmfsr {
namespace {

constexpr int MW = 64, MH = 32, THREADS = 256, PX = MH / 4;
constexpr int RAW_CAP = 3840;   // u16 Bayer footprint
constexpr int LUMA_CAP = 1024;  // quad sums
constexpr int OM_CAP = 800;     // Omega (3 x f64)
constexpr int RH_CAP = 640;     // R_hat window of the tile (base grid)
constexpr int VT_CAP = 640;     // tile displacements spanned by the tile
constexpr float SLACK = 64.f;   // log2 headroom above the reference exponent
// -log2(e) / 2: exponent of eq. (2) in base 2.
constexpr double NEG_HALF_LOG2E = -0.72134752044448170368;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ int colour_of(int col4, int parity) { return (col4 >> (2 * parity)) & 3; }

struct RowInfo {
  int ya, yb;  // R_hat window row offsets (already multiplied by the window width)
  float fy;
};

__global__ __launch_bounds__(THREADS) void k_merge(const uint16_t* __restrict__ frames,
                                                   const float* __restrict__ motion,
                                                   const float* __restrict__ rmin, Geometry g,
                                                   MergeConsts mc, float* __restrict__ out) {
  __shared__ double sY[MH];
  __shared__ int sTyRow[MH], sTxCol[MW];
  __shared__ RowInfo sRow[MH];
  __shared__ float2 sV[VT_CAP];
  __shared__ uint16_t sRaw[RAW_CAP];
  __shared__ int sLum[LUMA_CAP];
  __shared__ double sOm[3][OM_CAP];
  __shared__ float sRh[RH_CAP];
  __shared__ int sRed[8];
  __shared__ int sRh0[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int C0 = blockIdx.x * MW, R0 = blockIdx.y * MH;
  const int ncol = min(MW, g.OW - C0), nrow = min(MH, g.OH - R0);

  // ---- per-tile geometry ------------------------------------------------
  const int C = C0 + lane;
  const bool col_ok = lane < ncol;
  const double X = ((double)C + 0.5) / g.scale;  // base-frame position of the column
  if (tid < MW) sTxCol[tid] = col_ok ? min((int)floor(X) / g.T, g.TX - 1) : 0;
  if (tid >= 64 && tid < 64 + MH) {
    const int r = tid - 64;
    const double Y = ((double)(R0 + r) + 0.5) / g.scale;
    sY[r] = Y;
    sTyRow[r] = r < nrow ? min((int)floor(Y) / g.T, g.TY - 1) : 0;
  }
  __syncthreads();
  const int txA = sTxCol[0], txB = sTxCol[ncol - 1];
  const int tyA = sTyRow[0], tyB = sTyRow[nrow - 1];
  const int ntx = txB - txA + 1, nty = tyB - tyA + 1;
  // R_hat window on the base half-res grid: bilinear corners of X/2 - 1/2.
  if (tid == 0) {
    const double xf = ((double)C0 + 0.5) / g.scale, xl = ((double)(C0 + ncol - 1) + 0.5) / g.scale;
    const double yf = sY[0], yl = sY[nrow - 1];
    sRh0[0] = clampi((int)floor(xf * 0.5 - 0.5), 0, g.w - 1);
    sRh0[1] = clampi((int)floor(xl * 0.5 - 0.5) + 1, 0, g.w - 1);
    sRh0[2] = clampi((int)floor(yf * 0.5 - 0.5), 0, g.h - 1);
    sRh0[3] = clampi((int)floor(yl * 0.5 - 0.5) + 1, 0, g.h - 1);
  }
  __syncthreads();
  const int rhc0 = sRh0[0], rhw = sRh0[1] - sRh0[0] + 1;
  const int rhr0 = sRh0[2], rhn = rhw * (sRh0[3] - sRh0[2] + 1);
  if (tid < MH) {
    const double hy = sY[tid] * 0.5 - 0.5;
    const double fhy = floor(hy);
    const int y0 = (int)fhy;
    RowInfo ri;
    ri.ya = (clampi(y0, 0, g.h - 1) - rhr0) * rhw;
    ri.yb = (clampi(y0 + 1, 0, g.h - 1) - rhr0) * rhw;
    ri.fy = (float)(hy - fhy);
    sRow[tid] = ri;
  }
  int rxa, rxb;
  float rfx;
  {
    const double hx = X * 0.5 - 0.5;
    const double fhx = floor(hx);
    rxa = clampi((int)fhx, 0, g.w - 1) - rhc0;
    rxb = clampi((int)fhx + 1, 0, g.w - 1) - rhc0;
    rfx = (float)(hx - fhx);
  }
  const int txl = sTxCol[lane] - txA;

  // ---- accumulators -----------------------------------------------------
  float num[PX][3], den[PX][3], M[PX][3];
#pragma unroll
  for (int p = 0; p < PX; ++p)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      num[p][c] = 0.f;
      den[p][c] = 0.f;
      M[p][c] = -INFINITY;
    }

  for (int fi = 0; fi < g.n; ++fi) {
    const int n = fi == 0 ? g.ref : (fi <= g.ref ? fi - 1 : fi);
    const bool is_ref = n == g.ref;
    const uint16_t* f = frames + (size_t)n * g.H * g.W;
    __syncthreads();
    for (int k = tid; k < nty * ntx; k += THREADS) {
      float2 v = make_float2(0.f, 0.f);
      if (!is_ref) {
        const float* p = motion + (((size_t)n * g.TY + tyA + k / ntx) * g.TX + txA + k % ntx) * 2;
        v = make_float2(p[0], p[1]);
      }
      sV[k] = v;
    }
    if (!is_ref) {
      const float* rm = rmin + (size_t)n * g.h * g.w;
      for (int k = tid; k < rhn; k += THREADS)
        sRh[k] = rm[(size_t)(rhr0 + k / rhw) * g.w + rhc0 + k % rhw];
    }

    // Segments: the whole tile, or one alignment tile at a time.
    bool whole = true;
    int seg = 0;
    while (true) {
      const int sty = whole ? -1 : seg / ntx, stx = whole ? -1 : seg % ntx;
      __syncthreads();
      if (tid < 8) sRed[tid] = 0x7fffffff;
      __syncthreads();
      // footprint bounds over the segment's pixels
      int b[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) b[q] = 0x7fffffff;
      if (col_ok) {
#pragma unroll
        for (int p = 0; p < PX; ++p) {
          const int r = wave * PX + p;
          if (r >= nrow) continue;
          const int tyl = sTyRow[r] - tyA;
          if (!whole && (tyl != sty || txl != stx)) continue;
          const float2 v = sV[tyl * ntx + txl];
          const double px = fmin(fmax(X + (double)v.x, -4.0), (double)g.W + 4.0);
          const double py = fmin(fmax(sY[r] + (double)v.y, -4.0), (double)g.H + 4.0);
          const int jc = (int)floor(px), ic = (int)floor(py);
          const int hj = (int)floor(px * 0.5 - 0.5), hi = (int)floor(py * 0.5 - 0.5);
          b[0] = min(b[0], jc); b[1] = min(b[1], -jc);
          b[2] = min(b[2], ic); b[3] = min(b[3], -ic);
          b[4] = min(b[4], hj); b[5] = min(b[5], -hj);
          b[6] = min(b[6], hi); b[7] = min(b[7], -hi);
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) b[q] = wave_min(b[q]);
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) atomicMin(&sRed[q], b[q]);
      }
      __syncthreads();
      const int jcmin = sRed[0], jcmax = -sRed[1], icmin = sRed[2], icmax = -sRed[3];
      const int hjmin = sRed[4], hjmax = -sRed[5], himin = sRed[6], himax = -sRed[7];
      const bool empty = jcmin > jcmax;
      // Omega window (bilinear corners), luma window (3x3 tensor border), raw window
      const int oc0 = clampi(hjmin, 0, g.w - 1), oc1 = clampi(hjmax + 1, 0, g.w - 1);
      const int or0 = clampi(himin, 0, g.h - 1), or1 = clampi(himax + 1, 0, g.h - 1);
      const int lc0 = max(oc0 - 1, 0), lc1 = min(oc1 + 1, g.w - 1);
      const int lr0 = max(or0 - 1, 0), lr1 = min(or1 + 1, g.h - 1);
      const int rc0 = min(2 * lc0, clampi(jcmin - 1, 0, g.W - 1));
      const int rc1 = max(2 * lc1 + 1, clampi(jcmax + 1, 0, g.W - 1));
      const int rr0 = min(2 * lr0, clampi(icmin - 1, 0, g.H - 1));
      const int rr1 = max(2 * lr1 + 1, clampi(icmax + 1, 0, g.H - 1));
      const int ow = oc1 - oc0 + 1, on = ow * (or1 - or0 + 1);
      const int lw = lc1 - lc0 + 1, ln = lw * (lr1 - lr0 + 1);
      const int rw = rc1 - rc0 + 1, rn = rw * (rr1 - rr0 + 1);
      if (!empty && whole && (on > OM_CAP || ln > LUMA_CAP || rn > RAW_CAP)) {
        whole = false;
        seg = 0;
        continue;
      }
      if (!empty) {
        // 3. stage raw footprint, quad sums, Omega
        for (int k = tid; k < rn; k += THREADS)
          sRaw[k] = f[(size_t)(rr0 + k / rw) * g.W + rc0 + k % rw];
        __syncthreads();
        for (int k = tid; k < ln; k += THREADS) {
          const int o = (2 * (lr0 + k / lw) - rr0) * rw + 2 * (lc0 + k % lw) - rc0;
          sLum[k] = (int)sRaw[o] + (int)sRaw[o + 1] + (int)sRaw[o + rw] + (int)sRaw[o + rw + 1];
        }
        __syncthreads();
        for (int k = tid; k < on; k += THREADS) {
          const int I = or0 + k / ow, J = oc0 + k % ow;
          int l[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
              l[a][bb] = sLum[(clampi(I + a - 1, 0, g.h - 1) - lr0) * lw + clampi(J + bb - 1, 0, g.w - 1) - lc0];
          double oxx, oxy, oyy;
          omega_from_quads(l, mc.om, oxx, oxy, oyy);
          sOm[0][k] = oxx;
          sOm[1][k] = oxy;
          sOm[2][k] = oyy;
        }
        __syncthreads();

        // 4. accumulate
        if (col_ok) {
#pragma unroll
          for (int p = 0; p < PX; ++p) {
            const int r = wave * PX + p;
            if (r >= nrow) continue;
            const int tyl = sTyRow[r] - tyA;
            if (!whole && (tyl != sty || txl != stx)) continue;
            float rho = 1.f;
            if (!is_ref) {
              const RowInfo ri = sRow[r];
              const float top = (1.f - rfx) * sRh[ri.ya + rxa] + rfx * sRh[ri.ya + rxb];
              const float bot = (1.f - rfx) * sRh[ri.yb + rxa] + rfx * sRh[ri.yb + rxb];
              rho = (1.f - ri.fy) * top + ri.fy * bot;
              if (!(rho > 0.f)) continue;
            }
            const float2 v = sV[tyl * ntx + txl];
            const double px = fmin(fmax(X + (double)v.x, -4.0), (double)g.W + 4.0);
            const double py = fmin(fmax(sY[r] + (double)v.y, -4.0), (double)g.H + 4.0);
            const double fjc = floor(px), fic = floor(py);
            const int jc = (int)fjc, ic = (int)fic;
            // Omega at p / 2 - 1/2 (bilinear, edge-clamped)
            const double hx = px * 0.5 - 0.5, hy = py * 0.5 - 0.5;
            const double fhj = floor(hx), fhi = floor(hy);
            const double fx = hx - fhj, fy = hy - fhi;
            const int hj = (int)fhj, hi = (int)fhi;
            const int oa = clampi(hj, 0, g.w - 1) - oc0, ob = clampi(hj + 1, 0, g.w - 1) - oc0;
            const int ya = (clampi(hi, 0, g.h - 1) - or0) * ow, yb = (clampi(hi + 1, 0, g.h - 1) - or0) * ow;
            double O[3];
#pragma unroll
            for (int e = 0; e < 3; ++e) {
              const double top = (1.0 - fx) * sOm[e][ya + oa] + fx * sOm[e][ya + ob];
              const double bot = (1.0 - fx) * sOm[e][yb + oa] + fx * sOm[e][yb + ob];
              O[e] = (1.0 - fy) * top + fy * bot;
            }
            // eq. (2): log2 w = -1/2 log2(e) d^T Omega^-1 d
            const double sc = NEG_HALF_LOG2E / (O[0] * O[2] - O[1] * O[1]);
            const double qa = O[2] * sc, qb2 = -2.0 * O[1] * sc, qc = O[0] * sc;
            double dx[3], dy[3], ax[3], cy[3], by[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              dx[j] = ((double)(jc + j - 1) + 0.5) - px;
              dy[j] = ((double)(ic + j - 1) + 0.5) - py;
              ax[j] = qa * dx[j] * dx[j];
              cy[j] = qc * dy[j] * dy[j];
              by[j] = qb2 * dy[j];
            }
            double E[3][3];
            float val[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              const int qi = ic + i - 1;
              const bool row_in = qi >= 0 && qi < g.H;
              const int lrow = (clampi(qi, rr0, rr1) - rr0) * rw;
#pragma unroll
              for (int j = 0; j < 3; ++j) {
                const int qj = jc + j - 1;
                const bool in = row_in && qj >= 0 && qj < g.W;
                E[i][j] = in ? (ax[j] + cy[i]) + by[i] * dx[j] : -INFINITY;
                val[i][j] = (float)sRaw[lrow + clampi(qj, rc0, rc1) - rc0];
              }
            }
            // Colour groups of the 3x3 window: centre, left/right, up/down, corners.
            const int pr = ic & 1, pc = jc & 1;
            const int c0 = colour_of(mc.col4, pr * 2 + pc);
            const int c1 = colour_of(mc.col4, pr * 2 + (pc ^ 1));
            const bool isG = c0 == 1;
            const int cX = isG ? c1 : c0;  // the R or B group that is not "other"
            const bool xIsR = cX == 0;
            const float m0 = (float)E[1][1];
            const float m1 = (float)fmax(E[1][0], E[1][2]);
            const float m2 = (float)fmax(E[0][1], E[2][1]);
            const float m3 = (float)fmax(fmax(E[0][0], E[0][2]), fmax(E[2][0], E[2][2]));
            const float fG = isG ? fmaxf(m0, m3) : fmaxf(m1, m2);
            const float fX = isG ? m1 : m0, fY = isG ? m2 : m3;
            const float fR = xIsR ? fX : fY, fB = xIsR ? fY : fX;
            if (fR > M[p][0] + SLACK || fG > M[p][1] + SLACK || fB > M[p][2] + SLACK) {
              const float fm[3] = {fR, fG, fB};
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                const float nm = fmaxf(M[p][c], fm[c]);
                if (nm > M[p][c]) {
                  const float s = __builtin_amdgcn_exp2f(M[p][c] - nm);
                  num[p][c] *= s;
                  den[p][c] *= s;
                  M[p][c] = nm;
                }
              }
            }
            const float MX = xIsR ? M[p][0] : M[p][2], MY = xIsR ? M[p][2] : M[p][0], MG = M[p][1];
            const double g0 = (double)(isG ? MG : MX), g1 = (double)(isG ? MX : MG);
            const double g2 = (double)(isG ? MY : MG), g3 = (double)(isG ? MG : MY);
            const float w11 = __builtin_amdgcn_exp2f((float)(E[1][1] - g0));
            const float w10 = __builtin_amdgcn_exp2f((float)(E[1][0] - g1));
            const float w12 = __builtin_amdgcn_exp2f((float)(E[1][2] - g1));
            const float w01 = __builtin_amdgcn_exp2f((float)(E[0][1] - g2));
            const float w21 = __builtin_amdgcn_exp2f((float)(E[2][1] - g2));
            const float w00 = __builtin_amdgcn_exp2f((float)(E[0][0] - g3));
            const float w02 = __builtin_amdgcn_exp2f((float)(E[0][2] - g3));
            const float w20 = __builtin_amdgcn_exp2f((float)(E[2][0] - g3));
            const float w22 = __builtin_amdgcn_exp2f((float)(E[2][2] - g3));
            const float S0n = w11 * val[1][1], S0d = w11;
            const float S1n = w10 * val[1][0] + w12 * val[1][2], S1d = w10 + w12;
            const float S2n = w01 * val[0][1] + w21 * val[2][1], S2d = w01 + w21;
            const float S3n = (w00 * val[0][0] + w02 * val[0][2]) + (w20 * val[2][0] + w22 * val[2][2]);
            const float S3d = (w00 + w02) + (w20 + w22);
            const float Gn = isG ? S0n + S3n : S1n + S2n, Gd = isG ? S0d + S3d : S1d + S2d;
            const float Xn = isG ? S1n : S0n, Xd = isG ? S1d : S0d;
            const float Yn = isG ? S2n : S3n, Yd = isG ? S2d : S3d;
            num[p][0] += rho * (xIsR ? Xn : Yn);
            den[p][0] += rho * (xIsR ? Xd : Yd);
            num[p][1] += rho * Gn;
            den[p][1] += rho * Gd;
            num[p][2] += rho * (xIsR ? Yn : Xn);
            den[p][2] += rho * (xIsR ? Yd : Xd);
          }
        }
      }
      if (whole) break;
      if (++seg >= nty * ntx) break;
    }
  }

  // eq. (1): normalise and map raw units to [0, 1]
  if (col_ok) {
    const size_t plane = (size_t)g.OH * g.OW;
#pragma unroll
    for (int p = 0; p < PX; ++p) {
      const int r = wave * PX + p;
      if (r >= nrow) continue;
      const size_t o = (size_t)(R0 + r) * g.OW + C;
#pragma unroll
      for (int c = 0; c < 3; ++c) out[o + c * plane] = (num[p][c] / den[p][c] - mc.black) * mc.inv_range;
    }
  }
}

}  // namespace

hipError_t launch_merge(const Geometry& g, const MergeConsts& mc, const uint16_t* frames,
                        const float* motion, const float* rmin, float* out, hipStream_t stream) {
  const dim3 grid((g.OW + MW - 1) / MW, (g.OH + MH - 1) / MH);
  hipLaunchKernelGGL(k_merge, grid, dim3(THREADS), 0, stream, frames, motion, rmin, g, mc, out);
  return hipGetLastError();
}

}  // namespace hmfsr
