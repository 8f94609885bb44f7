// Host replay of the merge kernels' per-frame window arithmetic (the shared
// header's footprint(), make_win() and samples_outside(), compiled for the
// CPU) over extreme displacement fields. For every output tile of the
// forward's tile shapes (64 x 16, 64 x 32) and the adjoint's (64 x 8) it
// checks that
//   * one alignment tile's windows always fit the LDS caps (the per-tile
//     fallback relies on it),
//   * the windows the kernel uses (the whole tile's when it fits, else each
//     alignment tile's) hold every sample, Omega corner, luma neighbour and
//     raw quad that a pixel which is not skipped reads.
// Prints "OK <pixels checked>" and exits 0, or names the first violation and
// exits 1.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <random>
#include <vector>

#include "../paper_1905_03277_amd/csrc/merge_common.h"

using namespace hmfsr;

namespace {

long long g_checked = 0;

bool fail(const char* what, const Geometry& g, int MH, int tx, int ty, int a, int b) {
  printf("FAIL %s: W=%d H=%d T=%d s=%.3f MH=%d tile (%d,%d) values %d %d\n", what, g.W, g.H, g.T, g.scale, MH, tx,
         ty, a, b);
  return false;
}

bool inside(int v, int lo, int n) { return v >= lo && v < lo + n; }

// Every entry a window set reads for its own layout: luma neighbours of each
// Omega entry, raw quads of each luma entry.
bool window_consistent(const Win& w, const Geometry& g, int MH, int tx, int ty) {
  for (int r = 0; r < w.oh; ++r)
    for (int c = 0; c < w.ow; ++c) {
      const int I = clampi(w.or0 + r, 0, g.h - 1), J = clampi(w.oc0 + c, 0, g.w - 1);
      if (!inside(I - 1, w.lr0, w.lh) || !inside(I + 1, w.lr0, w.lh)) return fail("luma rows", g, MH, tx, ty, I, w.lr0);
      if (!inside(J - 1, w.lc0, w.lw) || !inside(J + 1, w.lc0, w.lw)) return fail("luma cols", g, MH, tx, ty, J, w.lc0);
    }
  for (int r = 0; r < w.lh; ++r)
    for (int c = 0; c < w.lw; ++c) {
      const int I = clampi(w.lr0 + r, 0, g.h - 1), J = clampi(w.lc0 + c, 0, g.w - 1);
      if (!inside(2 * I, w.rr0, w.rh) || !inside(2 * I + 1, w.rr0, w.rh)) return fail("raw rows", g, MH, tx, ty, I, w.rr0);
      if (!inside(2 * J, w.rc0, w.rw) || !inside(2 * J + 1, w.rc0, w.rw)) return fail("raw cols", g, MH, tx, ty, J, w.rc0);
    }
  return true;
}

// What one pixel at base position (X, Y) displaced by v reads from window w.
bool pixel_covered(double X, double Y, float vx, float vy, const Win& w, const Geometry& g, int MH, int tx, int ty) {
  const double px = X + (double)vx, py = Y + (double)vy;
  const int jc = (int)floor(px), ic = (int)floor(py);
  if (samples_outside(jc, ic, g)) return true;
  ++g_checked;
  if (!inside(ic - 1, w.rr0, w.rh) || !inside(ic + 1, w.rr0, w.rh)) return fail("sample rows", g, MH, tx, ty, ic, w.rr0);
  if (!inside(jc - 1, w.rc0, w.rw) || !inside(jc + 1, w.rc0, w.rw)) return fail("sample cols", g, MH, tx, ty, jc, w.rc0);
  const int hj = (int)floor(px * 0.5 - 0.5), hi = (int)floor(py * 0.5 - 0.5);
  if (!inside(hj, w.oc0, w.ow) || !inside(hj + 1, w.oc0, w.ow)) return fail("Omega cols", g, MH, tx, ty, hj, w.oc0);
  if (!inside(hi, w.or0, w.oh) || !inside(hi + 1, w.or0, w.oh)) return fail("Omega rows", g, MH, tx, ty, hi, w.or0);
  return true;
}

template <int MH>
bool check_tiles(const Geometry& g, const std::vector<float>& mo) {
  using CP = Caps<MH>;
  const float vlim = (float)(std::max(g.W, g.H) + 16);
  const int tiles_x = (g.OW + MW - 1) / MW, tiles_y = (g.OH + MH - 1) / MH;
  for (int ty = 0; ty < tiles_y; ++ty)
    for (int tx = 0; tx < tiles_x; ++tx) {
      const int C0 = tx * MW, R0 = ty * MH;
      const int ncol = std::min(MW, g.OW - C0), nrow = std::min(MH, g.OH - R0);
      std::vector<double> X(ncol), Y(nrow);
      std::vector<int> tcol(ncol), trow(nrow);
      for (int c = 0; c < ncol; ++c) {
        X[c] = out_pos(C0 + c, g.scale);
        tcol[c] = tile_of(X[c], g.T, g.TX);
      }
      for (int r = 0; r < nrow; ++r) {
        Y[r] = out_pos(R0 + r, g.scale);
        trow[r] = tile_of(Y[r], g.T, g.TY);
      }
      const int txA = tcol[0], tyA = trow[0];
      const int ntx = tcol[ncol - 1] - txA + 1, nty = trow[nrow - 1] - tyA + 1;
      if (ntx > CP::TX || nty > CP::TY) return fail("alignment tiles per output tile", g, MH, tx, ty, ntx, nty);
      std::vector<Win> tw(ntx * nty);
      std::vector<float> vx(ntx * nty), vy(ntx * nty);
      Bounds all = {1 << 30, -(1 << 30), 1 << 30, -(1 << 30), 1 << 30, -(1 << 30), 1 << 30, -(1 << 30)};
      for (int ky = 0; ky < nty; ++ky)
        for (int kx = 0; kx < ntx; ++kx) {
          int clo = ncol, chi = -1, rlo = nrow, rhi = -1;
          for (int c = 0; c < ncol; ++c)
            if (tcol[c] == txA + kx) { clo = std::min(clo, c); chi = c; }
          for (int r = 0; r < nrow; ++r)
            if (trow[r] == tyA + ky) { rlo = std::min(rlo, r); rhi = r; }
          const size_t t = ((size_t)(tyA + ky) * g.TX + txA + kx) * 2;
          const int k = ky * ntx + kx;
          // the kernels' clamp of the vector (non-finite values included)
          vx[k] = fminf(fmaxf(mo[t], -vlim), vlim);
          vy[k] = fminf(fmaxf(mo[t + 1], -vlim), vlim);
          const Bounds b = footprint(X[clo] + (double)vx[k], X[chi] + (double)vx[k], Y[rlo] + (double)vy[k],
                                     Y[rhi] + (double)vy[k], g);
          const Win w = make_win(b, g);
          if (w.rw * w.rh > CP::RAW) return fail("one tile's raw window", g, MH, tx, ty, w.rw, w.rh);
          if (w.lw * w.lh > CP::LUMA) return fail("one tile's luma window", g, MH, tx, ty, w.lw, w.lh);
          if (w.ow * w.oh > CP::OM) return fail("one tile's Omega window", g, MH, tx, ty, w.ow, w.oh);
          if (!window_consistent(w, g, MH, tx, ty)) return false;
          tw[k] = w;
          all.jc0 = std::min(all.jc0, b.jc0); all.jc1 = std::max(all.jc1, b.jc1);
          all.ic0 = std::min(all.ic0, b.ic0); all.ic1 = std::max(all.ic1, b.ic1);
          all.hj0 = std::min(all.hj0, b.hj0); all.hj1 = std::max(all.hj1, b.hj1);
          all.hi0 = std::min(all.hi0, b.hi0); all.hi1 = std::max(all.hi1, b.hi1);
        }
      const Win W = make_win(all, g);
      const bool whole = W.ow * W.oh <= CP::OM && W.lw * W.lh <= CP::LUMA && W.rw * W.rh <= CP::RAW;
      if (whole && !window_consistent(W, g, MH, tx, ty)) return false;
      for (int r = 0; r < nrow; ++r)
        for (int c = 0; c < ncol; ++c) {
          const int k = (trow[r] - tyA) * ntx + (tcol[c] - txA);
          if (!pixel_covered(X[c], Y[r], vx[k], vy[k], whole ? W : tw[k], g, MH, tx, ty)) return false;
        }
    }
  return true;
}

Geometry geometry(int W, int H, int T, double s) {
  Geometry g = {};
  g.W = W; g.H = H; g.w = W / 2; g.h = H / 2;
  g.T = T; g.TY = (H + T - 1) / T; g.TX = (W + T - 1) / T;
  g.OH = (int)floor(H * s + 0.5); g.OW = (int)floor(W * s + 0.5);
  g.scale = s;
  return g;
}

}  // namespace

int main() {
  std::mt19937_64 rng(190503277);
  const int sizes[][2] = {{256, 256}, {64, 48}, {200, 136}, {4, 4}, {96, 520}, {1024, 64}};
  const int tiles[] = {8, 16, 32, 64};
  const double scales[] = {1.0, 1.25, 1.5, 2.0, 3.0};
  const float specials[] = {0.f, 0.5f, -0.5f, 3.7f, -40.f, 200.f, -200.f, 400.f, -400.f, 1e6f, -1e9f,
                            INFINITY, -INFINITY, NAN};
  const int nspec = sizeof(specials) / sizeof(specials[0]);
  int cases = 0;
  for (auto& sz : sizes)
    for (int T : tiles)
      for (double s : scales) {
        const Geometry g = geometry(sz[0], sz[1], T, s);
        for (int field = 0; field < 6; ++field) {
          std::vector<float> mo((size_t)g.TY * g.TX * 2);
          std::uniform_real_distribution<float> wide(-(float)(g.W + 64), (float)(g.W + 64));
          for (size_t i = 0; i < mo.size(); ++i) {
            switch (field) {
              case 0: mo[i] = specials[rng() % nspec]; break;            // mixed extremes
              case 1: mo[i] = wide(rng); break;                           // anywhere in and around the frame
              case 2: mo[i] = (i & 1) ? 0.f : ((i / 2) % 2 ? 400.f : -400.f); break;  // alternating jumps
              case 3: mo[i] = 200.f + (float)(rng() % 7) - 3.f; break;    // coherent, far right / down
              case 4: mo[i] = -200.f - (float)(rng() % 7); break;         // coherent, far left / up
              default: mo[i] = (float)((int)(rng() % 81) - 40) * 0.25f; break;  // moderate spread
            }
          }
          if (!check_tiles<16>(g, mo) || !check_tiles<32>(g, mo) || !check_tiles<8>(g, mo)) return 1;
          ++cases;
        }
      }
  printf("OK %lld pixels, %d fields\n", g_checked, cases);
  return 0;
}
