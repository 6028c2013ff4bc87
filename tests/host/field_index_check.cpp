// Host check of the field, link and clover-table index maps
// (paper_1103_1363_amd/csrc/field_index.h) on nblk 64-site blocks: every map
// is a bijection onto its buffer, and the maps that relate two layouts (an
// FP32 entry to its FP64 entry, a chunked FP32 clover entry to its FP64 one,
// the site of an FP32 entry) agree with the per-site maps.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1103_1363_amd/csrc/field_index.h"

using lq::SB;

static int fails = 0;
static void check(bool ok, const char* what, long long a, long long b) {
  if (!ok && fails++ < 10) std::printf("FAIL %s %lld %lld\n", what, a, b);
}

// each index in [0, n) hit exactly once
static void bijection(const std::vector<long long>& idx, long long n, const char* what) {
  std::vector<int> hit(n, 0);
  for (long long i : idx) {
    check(i >= 0 && i < n, what, i, n);
    if (i >= 0 && i < n) ++hit[i];
  }
  for (long long i = 0; i < n; ++i) check(hit[i] == 1, what, i, hit[i]);
}

int main(int argc, char** argv) {
  const long long nblk = argc > 1 ? std::atoll(argv[1]) : 3;
  const long long ns = nblk * SB;
  std::vector<long long> f16, f32, f64, c16, c32, c64, l16, l32, l64;
  for (long long s = 0; s < ns; ++s) {
    for (int c = 0; c < 12; ++c) {
      f16.push_back(lq::chunk16_idx(s, c >> 2) * 4 + (c & 3));  // 4-byte pairs
      const long long j = lq::chunk32_idx(s, c >> 1) * 2 + (c & 1);  // complex
      f32.push_back(j);
      f64.push_back(lq::spin_idx(s, c));
      check(lq::flat32_to_64(j) == lq::spin_idx(s, c), "flat32_to_64", j, s);
      check(lq::site_in_block32(j) == (int)(s & 63), "site_in_block32", j, s);
    }
    for (int e = 0; e < 36; ++e) {
      c16.push_back(lq::clov16_idx(s, e));
      c32.push_back(lq::clov32_idx(s, e));
      c64.push_back(lq::clov_idx(s, e));
      check(lq::clov32_to_64(lq::clov32_idx(s, e)) == lq::clov_idx(s, e), "clov32_to_64", s, e);
    }
    for (int p = 0; p < 2; ++p)
      for (int mu = 0; mu < 4; ++mu)
        for (int c = 0; c < 6; ++c) {
          l16.push_back(lq::link16_idx(nblk, p, mu, s, c));
          l32.push_back(lq::link32_idx(nblk, p, mu, s, c));
          l64.push_back(lq::link_idx(nblk, p, mu, s, c));
        }
  }
  bijection(f16, ns * 12, "fp16 spinor");
  bijection(f32, ns * 12, "fp32 spinor");
  bijection(f64, ns * 12, "fp64 spinor");
  bijection(c16, ns * 36, "fp16 clover");
  bijection(c32, ns * 36, "fp32 clover");
  bijection(c64, ns * 36, "fp64 clover");
  bijection(l16, ns * 48, "fp16 links");
  bijection(l32, ns * 48, "fp32 links");
  bijection(l64, ns * 48, "fp64 links");
  // 16-byte loads: the chunk of four FP16 pairs, two FP32 complex numbers,
  // four FP16 clover entries (k < 16 of a chirality block) and two FP32
  // ones start on a 16-byte boundary and are consecutive
  for (long long s = 0; s < ns; ++s) {
    for (int k = 0; k < 3; ++k) check(lq::chunk16_idx(s, k) * 4 % 4 == 0, "fp16 chunk", s, k);
    for (int b = 0; b < 2; ++b)
      for (int k = 0; k < 16; k += 4) {
        const long long i0 = lq::clov16_idx(s, 18 * b + k);
        check(i0 % 4 == 0, "fp16 clover chunk", s, k);
        for (int j = 1; j < 4; ++j) check(lq::clov16_idx(s, 18 * b + k + j) == i0 + j, "fp16 clover run", s, k);
      }
    for (int e = 0; e < 36; e += 2) {
      check(lq::clov32_idx(s, e) % 2 == 0, "fp32 clover chunk", s, e);
      check(lq::clov32_idx(s, e + 1) == lq::clov32_idx(s, e) + 1, "fp32 clover run", s, e);
    }
    for (int p = 0; p < 2; ++p)
      for (int mu = 0; mu < 4; ++mu) {
        const long long a = lq::link16_idx(nblk, p, mu, s, 0), b4 = lq::link16_idx(nblk, p, mu, s, 4);
        check(a % 4 == 0 && b4 % 2 == 0, "fp16 link chunks", s, mu);
        for (int c = 1; c < 4; ++c) check(lq::link16_idx(nblk, p, mu, s, c) == a + c, "fp16 link run", s, c);
        check(lq::link16_idx(nblk, p, mu, s, 5) == b4 + 1, "fp16 link tail", s, mu);
        for (int c = 0; c < 6; c += 2) {
          const long long x = lq::link32_idx(nblk, p, mu, s, c);
          check(x % 2 == 0 && lq::link32_idx(nblk, p, mu, s, c + 1) == x + 1, "fp32 link chunk", s, c);
        }
      }
  }
  std::printf(fails ? "FAIL\n" : "ok\n");
  return fails ? 1 : 0;
}
