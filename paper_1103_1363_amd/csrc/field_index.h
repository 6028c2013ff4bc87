// Index maps of the device fields, clover tables and links (element
// offsets inside the byte buffers the library allocates).
//
// Plain C++ (no device-only constructs) so that the host tests can compile
// it with g++; the HIP sources include it with LQ_HD = __host__ __device__.
#pragma once

#include <cstdint>

#ifndef LQ_HD
#define LQ_HD
#endif

namespace lq {

// ---------------------------------------------------------------- layout
// Sites of one parity are numbered by their checkerboard index s = i / 2
// (i the full-lattice index).  Device fields group sites into blocks of 64;
// in FP64 fields each complex component occupies 64 consecutive slots inside
// a block, so the 64 lanes of a wavefront read one component of 64
// consecutive sites with a single coalesced load (FP32 and FP16 fields:
// 16-byte chunks, below).
constexpr int SB = 64;  // sites per block

LQ_HD inline int64_t spin_idx(int64_t s, int c) {  // c in [0, 12)
  return ((s >> 6) * 12 + c) * SB + (s & 63);
}
// FP16 spinor fields are chunked instead: inside a block the 12 components of
// a site (4 bytes each) form three 16-byte chunks (components 4k .. 4k+3),
// and chunk k of the block's 64 sites is contiguous (1 KB).  A lane reads
// its site's spinor with three 16-byte loads, and a wavefront's load of one
// chunk of 64 consecutive sites is one coalesced kilobyte.  Index in 16-byte
// units, k in [0, 3).
LQ_HD inline int64_t chunk16_idx(int64_t s, int k) {
  return ((s >> 6) * 3 + k) * SB + (s & 63);
}
// FP32 spinor fields are chunked too: 16-byte chunks of two complex
// components (2k, 2k + 1), chunk k of the block's 64 sites contiguous.
// Index in 16-byte units, k in [0, 6).
LQ_HD inline int64_t chunk32_idx(int64_t s, int k) {
  return ((s >> 6) * 6 + k) * SB + (s & 63);
}
// Entrywise kernels that pair an FP32 field with an FP64 one: the FP64
// (component-major) entry that holds FP32 entry j (both counted in complex
// entries; a block is 768 entries in either precision), and the site within
// its block of an FP32 entry.
LQ_HD inline int64_t flat32_to_64(int64_t j) {
  const int64_t b = j / 768;
  const int r = (int)(j - b * 768);
  return b * 768 + ((r >> 7) * 2 + (r & 1)) * SB + ((r & 127) >> 1);
}
LQ_HD inline int site_in_block32(int64_t j) { return (int)((j & 127) >> 1); }
LQ_HD inline int64_t clov_idx(int64_t s, int c) {  // c in [0, 36)
  return ((s >> 6) * 36 + c) * SB + (s & 63);
}
// Clover tables in FP32 and FP16 are chunked for 16-byte loads too.  FP32:
// chunks of two entries (2j, 2j + 1), chunk j of the block's 64 sites
// contiguous, index in complex units.  FP16: per chirality block b (entries
// 18 b .. 18 b + 17) the entries 0..15 as four 16-byte chunks and 16, 17 as
// one 8-byte chunk, index in 4-byte pairs.  e in [0, 36).
LQ_HD inline int64_t clov32_idx(int64_t s, int e) {
  return ((s >> 6) * 18 + (e >> 1)) * (2 * SB) + (s & 63) * 2 + (e & 1);
}
LQ_HD inline int64_t clov16_idx(int64_t s, int e) {
  const int b = e >= 18 ? 1 : 0, k = e - 18 * b;
  const int64_t base = (s >> 6) * (36 * SB) + b * (18 * SB);
  return k < 16 ? base + (k >> 2) * (4 * SB) + (s & 63) * 4 + (k & 3)
                : base + 16 * SB + (s & 63) * 2 + (k - 16);
}
// compressed links: parity p, direction mu, site s, complex entry c in [0, 6)
// (row 0 then row 1)
LQ_HD inline int64_t link_idx(int64_t nblk, int p, int mu, int64_t s, int c) {
  return ((((int64_t)p * 4 + mu) * nblk + (s >> 6)) * 6 + c) * SB + (s & 63);
}
// FP32 links: per (parity, mu, block) three 16-byte chunks of two entries
// (entries 2k, 2k + 1), chunk k of the 64 sites contiguous; index of entry c
// in complex (8-byte) units.
LQ_HD inline int64_t link32_idx(int64_t nblk, int p, int mu, int64_t s, int c) {
  return (((int64_t)p * 4 + mu) * nblk + (s >> 6)) * 384 + (c >> 1) * 128 + (s & 63) * 2 + (c & 1);
}
// FP16 links are chunked like FP16 spinors: per (parity, mu, block) the
// entries 0..3 of the 64 sites as 16-byte chunks (1 KB), then entries 4, 5 as
// 8-byte chunks (512 B); index of entry c in 4-byte pairs.
LQ_HD inline int64_t link16_idx(int64_t nblk, int p, int mu, int64_t s, int c) {
  const int64_t base = (((int64_t)p * 4 + mu) * nblk + (s >> 6)) * 384;
  return c < 4 ? base + (s & 63) * 4 + c : base + 256 + (s & 63) * 2 + (c - 4);
}

// The FP64 clover-table entry that holds entry i of a chunked FP32 table
// (both in complex units; a block holds 36 x 64 entries in either form).
LQ_HD inline int64_t clov32_to_64(int64_t i) {
  const int64_t blk = i / (36 * SB);
  const int r = (int)(i - blk * (36 * SB));
  return (blk * 36 + 2 * (r >> 7) + (r & 1)) * SB + ((r & 127) >> 1);
}

}  // namespace lq
