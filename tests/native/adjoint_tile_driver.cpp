// Host driver: the reverse of a 2D operator as the GPU runs it (three
// cotangent stages fused over tiles, their intermediate values in a block's
// shared memory) against the same reverse stated as three passes over
// whole grids (rv_tc, rv_pred, rv_prim), on seeded random states, output
// cotangents and coefficient accumulators.  Every block is emulated phase
// by phase in the order its barriers impose; the tile's shared memory
// starts as NaN, so a read of a slot no stage wrote shows in the result.
// Results must agree bit for bit (Xb, MU, KB) over both axes, both plate
// closures, the TVD term on and off, Courant numbers on both sides of the
// limiter's knee, and grids narrower than a tile (the periodic x direction
// wraps inside one region) or with ragged last tiles.
#define MTVD_HD
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "mtvd_adjoint.h"

using namespace mtvd::adj;

int main() {
  int bad = 0, runs = 0;
  for (int axis : {0, 2})
    for (int wo : {1, 2})
      for (int tvd : {0, 1})
        for (int nx : {8, 13, 30})
          for (int nz : {5, 6, 9, 17, 30})
            for (int seed = 0; seed < 2; ++seed) {
              std::mt19937_64 g(seed * 100003ULL + nz * 101 + nx * 7 + axis + wo * 3 + tvd * 11);
              std::uniform_real_distribution<double> u(-1.0, 1.0), up(0.5, 2.0);
              AC c{};
              c.nx = nx;
              c.nz = nz;
              c.M = nz - 1;
              c.axis = axis;
              c.cnt = (long long)nx * nz;
              c.ihx = 1 / 0.1;
              c.ihz = 1 / 0.15;
              c.iha = axis == 0 ? c.ihx : c.ihz;
              c.cv = 2.5;
              c.icv = 0.4;
              c.a = 1.0;
              c.gam_a = 1.4;
              c.g = 0.3;
              c.mu = 0.01;
              c.K = 0.02;
              c.lam = -2.0 / 3;
              c.Tb = 1.0;
              c.Tt = 0.5;
              c.tau = 0.01;
              c.lm = 0.02 + 0.5 * seed;   // Courant numbers below and above 1/2
              c.wall_order = wo;
              c.tvd_on = tvd;
              const long long cnt = c.cnt;
              std::vector<double> zr(nz), X(4 * cnt), P(4 * cnt), S(cnt), XP(4 * cnt), PP(4 * cnt),
                  Yb(4 * cnt), MU0(cnt), KB0(cnt);
              for (int k = 0; k < nz; ++k) zr[k] = k / (double)(nz - 1);
              for (long long n = 0; n < cnt; ++n) {
                X[n] = up(g);
                X[cnt + n] = 0.3 * u(g);
                X[2 * cnt + n] = 0.3 * u(g);
                X[3 * cnt + n] = 5 + up(g);
                for (int q = 0; q < 4; ++q) Yb[q * cnt + n] = u(g);
                MU0[n] = u(g);
                KB0[n] = u(g);
              }
              // some equal neighbours: TVD faces with no jump
              for (long long n = 0; n + 1 < cnt; n += 5)
                for (int q = 0; q < 4; ++q) X[q * cnt + n] = X[q * cnt + n + 1];
              Arr F{};
              F.X = X.data();
              F.zr = zr.data();
              F.P = P.data();
              F.S = S.data();
              F.XP = XP.data();
              F.PP = PP.data();
              for (int k = 0; k < nz; ++k)
                for (int i = 0; i < nx; ++i) fw_all(c, F, i, k);
              // three passes over the grid
              std::vector<double> gXb(4 * cnt), gXPb(4 * cnt), gPPb(4 * cnt), gDPb(5 * cnt),
                  gPB(4 * cnt), gDB(5 * cnt), gSB(cnt), gMU = MU0, gKB = KB0;
              Arr G = F;
              G.Yb = Yb.data();
              G.Xb = gXb.data();
              G.XPb = gXPb.data();
              G.PPb = gPPb.data();
              G.DPb = gDPb.data();
              G.PB = gPB.data();
              G.DB = gDB.data();
              G.SB = gSB.data();
              G.MU = gMU.data();
              G.KB = gKB.data();
              for (int k = 0; k < nz; ++k)
                for (int i = 0; i < nx; ++i) rv_tc(c, G, i, k);
              for (int k = 0; k < nz; ++k)
                for (int i = 0; i < nx; ++i) rv_pred(c, G, i, k);
              for (int k = 0; k < nz; ++k)
                for (int i = 0; i < nx; ++i) rv_prim(c, G, i, k);
              // fused tiles, block by block
              std::vector<double> tXb(4 * cnt, NAN), tMU = MU0, tKB = KB0;
              Arr T = F;
              T.Yb = Yb.data();
              T.Xb = tXb.data();
              T.MU = tMU.data();
              T.KB = tKB.data();
              const int na = axis == 0 ? nx : nz, nb = axis == 0 ? nz : nx;
              for (int a0 = 0; a0 < na; a0 += kTA)
                for (int b0 = 0; b0 < nb; b0 += kTB) {
                  std::vector<double> L(kTileDoubles, NAN);
                  std::vector<PredOut> po(kNP);
                  std::vector<char> put(kNP);
                  for (int t = 0; t < kNT; ++t) tile_tc(c, T, L.data(), a0, b0, t);
                  for (int t = 0; t < kNP; ++t) put[t] = tile_pred(c, T, L.data(), a0, b0, t, po[t]);
                  for (int t = 0; t < kNP; ++t)
                    if (put[t]) tile_pred_put(L.data(), t, po[t]);
                  for (int t = 0; t < kNO; ++t) tile_prim(c, T, L.data(), a0, b0, t);
                }
              ++runs;
              auto same = [&](const std::vector<double>& x, const std::vector<double>& y,
                              const char* what) {
                if (memcmp(x.data(), y.data(), x.size() * sizeof(double))) {
                  ++bad;
                  printf("differ: %s axis %d wall_order %d tvd %d nx %d nz %d seed %d\n", what, axis,
                         wo, tvd, nx, nz, seed);
                }
              };
              same(tXb, gXb, "Xb");
              same(tMU, gMU, "MU");
              same(tKB, gKB, "KB");
            }
  printf("%d cases, %d differ\n", runs, bad);
  if (bad) return 1;
  printf("adjoint tile driver ok\n");
  return 0;
}
