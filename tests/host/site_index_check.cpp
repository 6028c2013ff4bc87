// Host check of the device site numbering (paper_1103_1363_amd/csrc/site_index.h):
// for each lattice given on the command line (Lx Ly Lz Lt target), every
// (parity, site) maps to coordinates of that parity and back, every
// coordinate is hit once, and the chosen tiles are even divisors.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1103_1363_amd/csrc/site_index.h"

int main(int argc, char** argv) {
  if ((argc - 1) % 5 != 0 || argc == 1) {
    std::fprintf(stderr, "usage: Lx Ly Lz Lt target ...\n");
    return 2;
  }
  for (int a = 1; a < argc; a += 5) {
    lq::Geo g{};
    for (int k = 0; k < 4; ++k) g.L[k] = std::atoi(argv[a + k]);
    const long long target = std::atoll(argv[a + 4]);
    lq::choose_tiles(g.L, target, g.T);
    lq::geo_finish(g);
    for (int k = 0; k < 4; ++k)
      if (g.T[k] < 2 || g.T[k] % 2 || g.L[k] % g.T[k]) {
        std::printf("FAIL tile %d %d %d %d\n", g.T[0], g.T[1], g.T[2], g.T[3]);
        return 1;
      }
    if (g.tvh > target && g.vh > target) {
      std::printf("FAIL tile too large\n");
      return 1;
    }
    const long long V = 2 * g.vh;
    std::vector<int> seen(V, 0);
    for (int p = 0; p < 2; ++p)
      for (long long s = 0; s < g.vh; ++s) {
        int x[4];
        lq::site_coords(g, p, s, x);
        for (int k = 0; k < 4; ++k)
          if (x[k] < 0 || x[k] >= g.L[k]) {
            std::printf("FAIL coords out of range\n");
            return 1;
          }
        if (((x[0] + x[1] + x[2] + x[3]) & 1) != p || lq::cb_index(g, x) != s) {
          std::printf("FAIL round trip p=%d s=%lld\n", p, s);
          return 1;
        }
        int l[4], tc[4];
        lq::site_local(g, p, s, l, tc);
        for (int k = 0; k < 4; ++k)
          if (tc[k] * g.T[k] + l[k] != x[k]) {
            std::printf("FAIL local coordinates\n");
            return 1;
          }
        // the division-free neighbour steps against explicitly wrapped coordinates
        for (int mu = 0; mu < 4; ++mu)
          for (int fwd = 0; fwd < 2; ++fwd) {
            int y[4] = {x[0], x[1], x[2], x[3]};
            y[mu] = (y[mu] + (fwd ? 1 : -1) + g.L[mu]) % g.L[mu];
            if (lq::neighbour(g, s, l, tc, mu, fwd != 0) != lq::cb_index(g, y)) {
              std::printf("FAIL neighbour mu=%d fwd=%d p=%d s=%lld\n", mu, fwd, p, s);
              return 1;
            }
          }
        const long long i = (((long long)x[3] * g.L[2] + x[2]) * g.L[1] + x[1]) * g.L[0] + x[0];
        int y[4];
        lq::canonical_coords(g, i, y);
        for (int k = 0; k < 4; ++k)
          if (y[k] != x[k]) {
            std::printf("FAIL canonical coords\n");
            return 1;
          }
        seen[i] += 1;
      }
    for (long long i = 0; i < V; ++i)
      if (seen[i] != 1) {
        std::printf("FAIL coverage\n");
        return 1;
      }
    std::printf("ok %d %d %d %d tiles %d %d %d %d\n", g.L[0], g.L[1], g.L[2], g.L[3], g.T[0],
                g.T[1], g.T[2], g.T[3]);
  }
  return 0;
}
