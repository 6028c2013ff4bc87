// Lattice geometry and the site numbering of device fields.
//
// The lattice is cut into tiles of T0 x T1 x T2 x T3 sites (each extent even
// and dividing the lattice extent).  Sites of one parity are numbered tile by
// tile (tiles in x-fastest order), and inside a tile in x-fastest order with
// the parity halving the x coordinate.  A workgroup of consecutive sites thus
// covers a compact 4-D region, and all workgroups of one XCD walk whole
// tiles, so the neighbours a hopping sweep reads are mostly still in that
// XCD's L2.  Tiles equal to the whole lattice give the plain checkerboard
// order i / 2.
//
// Plain C++ (no device-only constructs) so that the host tests can compile
// it with g++; the HIP sources include it with LQ_HD = __host__ __device__.
#pragma once

#include <cstdint>

#ifndef LQ_HD
#define LQ_HD
#endif

namespace lq {

struct Geo {
  int L[4];      // lattice extents Lx, Ly, Lz, Lt
  int T[4];      // tile extents
  int NT[4];     // tiles per direction
  int txh;       // T[0] / 2
  int apt;       // fermion fields antiperiodic in t
  int64_t tvh;   // sites of one parity per tile
  int64_t vh;    // sites per parity
  int64_t nblk;  // blocks of 64 sites per parity (vh rounded up)
  int hs[4];     // site-number step of +1 in direction mu inside a tile (mu >= 1)
  int64_t ts[4]; // site-number step of +1 tile in direction mu
};

// Fill the derived fields of g from g.L and g.T.
inline void geo_finish(Geo& g) {
  int64_t tv = 1;
  for (int k = 0; k < 4; ++k) {
    g.NT[k] = g.L[k] / g.T[k];
    tv *= g.T[k];
  }
  g.txh = g.T[0] / 2;
  g.tvh = tv / 2;
  g.vh = (int64_t)g.L[0] * g.L[1] * g.L[2] * g.L[3] / 2;
  g.nblk = (g.vh + 63) / 64;
  g.hs[0] = 0;
  g.hs[1] = g.T[0] / 2;
  g.hs[2] = g.T[0] * g.T[1] / 2;
  g.hs[3] = g.T[0] * g.T[1] * g.T[2] / 2;
  g.ts[0] = g.tvh;
  g.ts[1] = g.tvh * g.NT[0];
  g.ts[2] = g.tvh * g.NT[0] * g.NT[1];
  g.ts[3] = g.tvh * g.NT[0] * g.NT[1] * g.NT[2];
}

// Site s of parity p: local coordinates inside its tile (l) and the tile's
// coordinates (tc); the lattice coordinate is tc * T + l.
LQ_HD inline void site_local(const Geo& g, int p, int64_t s, int l[4], int tc[4]) {
  const unsigned tile = (unsigned)(s / g.tvh);
  unsigned r = (unsigned)(s - (int64_t)tile * g.tvh);
  const unsigned xh = r % (unsigned)g.txh;
  r /= (unsigned)g.txh;
  l[1] = (int)(r % (unsigned)g.T[1]);
  r /= (unsigned)g.T[1];
  l[2] = (int)(r % (unsigned)g.T[2]);
  l[3] = (int)(r / (unsigned)g.T[2]);
  unsigned q = tile;
  tc[0] = (int)(q % (unsigned)g.NT[0]);
  q /= (unsigned)g.NT[0];
  tc[1] = (int)(q % (unsigned)g.NT[1]);
  q /= (unsigned)g.NT[1];
  tc[2] = (int)(q % (unsigned)g.NT[2]);
  tc[3] = (int)(q / (unsigned)g.NT[2]);
  // tile origins have even coordinates, so the parity fixes the low x bit
  l[0] = 2 * (int)xh + ((p + l[1] + l[2] + l[3]) & 1);
}

// Device number of the neighbour of site s (local coordinates l, tile
// coordinates tc) one step in direction mu, forward (fwd) or backward,
// periodic, without divisions.
// (Written with selects only: branches here split every hop into basic
// blocks and keep the compiler from interleaving loads and arithmetic.)
LQ_HD inline int64_t neighbour(const Geo& g, int64_t s, const int l[4], const int tc[4], int mu,
                               bool fwd) {
  const int T = g.T[mu];
  const bool edge = fwd ? (l[mu] + 1 == T) : (l[mu] == 0);  // the step leaves the tile
  const bool wrap = fwd ? (tc[mu] + 1 == g.NT[mu]) : (tc[mu] == 0);  // ... and the lattice
  const int64_t tstep = wrap ? (fwd ? -(int64_t)(g.NT[mu] - 1) : (int64_t)(g.NT[mu] - 1))
                             : (fwd ? 1 : -1);
  const int64_t dtile = edge ? tstep * g.ts[mu] : 0;
  int64_t dsite;
  if (mu == 0) {
    const int lx = l[0];
    const int in_step = fwd ? (lx & 1) : -(1 - (lx & 1));
    const int out_step = fwd ? -(lx >> 1) : ((T - 1) >> 1);
    dsite = edge ? out_step : in_step;
  } else {
    const int64_t h = g.hs[mu];
    dsite = edge ? (fwd ? -(int64_t)(T - 1) * h : (int64_t)(T - 1) * h) : (fwd ? h : -h);
  }
  return s + dtile + dsite;
}

// Coordinates of site s (device numbering) of parity p.
LQ_HD inline void site_coords(const Geo& g, int p, int64_t s, int x[4]) {
  const int64_t tile = s / g.tvh;
  int64_t r = s - tile * g.tvh;
  const int xh = (int)(r % g.txh);
  r /= g.txh;
  const int ly = (int)(r % g.T[1]);
  r /= g.T[1];
  const int lz = (int)(r % g.T[2]);
  const int lt = (int)(r / g.T[2]);
  int64_t q = tile;
  const int tx = (int)(q % g.NT[0]);
  q /= g.NT[0];
  const int ty = (int)(q % g.NT[1]);
  q /= g.NT[1];
  const int tz = (int)(q % g.NT[2]);
  const int tt = (int)(q / g.NT[2]);
  x[1] = ty * g.T[1] + ly;
  x[2] = tz * g.T[2] + lz;
  x[3] = tt * g.T[3] + lt;
  // tile origins have even coordinates, so the parity fixes the low x bit
  x[0] = tx * g.T[0] + 2 * xh + ((p + x[1] + x[2] + x[3]) & 1);
}

// Device number of the site at coordinates x (its parity is (sum x) & 1).
LQ_HD inline int64_t cb_index(const Geo& g, const int x[4]) {
  const int tx = x[0] / g.T[0], ty = x[1] / g.T[1], tz = x[2] / g.T[2], tt = x[3] / g.T[3];
  const int lx = x[0] - tx * g.T[0], ly = x[1] - ty * g.T[1], lz = x[2] - tz * g.T[2],
            lt = x[3] - tt * g.T[3];
  const int64_t tile = (((int64_t)tt * g.NT[2] + tz) * g.NT[1] + ty) * g.NT[0] + tx;
  const int64_t intra = (((int64_t)lt * g.T[2] + lz) * g.T[1] + ly) * g.T[0] + lx;
  return tile * g.tvh + (intra >> 1);
}

// Coordinates of the full-lattice canonical index i = ((x3 Lz + x2) Ly + x1) Lx + x0.
LQ_HD inline void canonical_coords(const Geo& g, int64_t i, int x[4]) {
  x[0] = (int)(i % g.L[0]);
  i /= g.L[0];
  x[1] = (int)(i % g.L[1]);
  i /= g.L[1];
  x[2] = (int)(i % g.L[2]);
  x[3] = (int)(i / g.L[2]);
}

// Tile extents for a lattice: every extent an even divisor of the lattice
// extent, half-tile volume at most `target` sites, minimal surface per
// volume (sum of 1/T), ties broken towards longer x rows.  A lattice whose
// half volume is within the target is a single tile.
inline void choose_tiles(const int L[4], int64_t target, int T[4]) {
  int best[4] = {L[0], L[1], L[2], L[3]};
  const int64_t vh = (int64_t)L[0] * L[1] * L[2] * L[3] / 2;
  if (vh <= target) {
    for (int k = 0; k < 4; ++k) T[k] = L[k];
    return;
  }
  double best_cost = 1e30;
  int best_tx = 0;
  bool found = false;
  for (int a = 2; a <= L[0]; a += 2) {
    if (L[0] % a) continue;
    for (int b = 2; b <= L[1]; b += 2) {
      if (L[1] % b) continue;
      for (int c = 2; c <= L[2]; c += 2) {
        if (L[2] % c) continue;
        for (int d = 2; d <= L[3]; d += 2) {
          if (L[3] % d) continue;
          const int64_t half = (int64_t)a * b * c * d / 2;
          if (half > target) continue;
          const double cost = 1.0 / a + 1.0 / b + 1.0 / c + 1.0 / d;
          if (!found || cost < best_cost - 1e-12 || (cost < best_cost + 1e-12 && a > best_tx)) {
            best_cost = cost;
            best_tx = a;
            best[0] = a, best[1] = b, best[2] = c, best[3] = d;
            found = true;
          }
        }
      }
    }
  }
  for (int k = 0; k < 4; ++k) T[k] = best[k];
}

}  // namespace lq
