// Tiling of a context and the tile tuner.
//
// A context numbers the sites of each parity inside 4-D tiles (the
// single-RHS fields, `geo`) and, separately, inside smaller tiles for the
// multi-RHS fields (`mr_geo`): within a tile the y, z and t neighbours of a
// wavefront's 64 sites are 64 consecutive sites, and the tile's extent sets
// how far a neighbour across it lies in memory, against what each XCD's L2
// holds.  lq_set_tiling changes the largest tile (sites of one parity) of
// either numbering before any field is laid out; lq_tune_tiles times the
// Schur operator for each candidate on a scratch context with unit links
// (the kernels' work does not depend on the link values) and keeps the
// fastest, cached in a JSON file per (GPU architecture, lattice, precision,
// right-hand sides).
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "lq_internal.h"

namespace {

std::string g_tune_error;

const char* prec_label(int p) {
  return p == LQ_F64 ? "f64" : p == LQ_F32 ? "f32" : p == LQ_F16 ? "f16" : "f16x";
}

std::string gpu_arch() {
  int dev = 0;
  LQ_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  LQ_HIP(hipGetDeviceProperties(&prop, dev));
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string tune_key(const int dims[4], int prec, int nrhs) {
  std::ostringstream k;
  k << gpu_arch() << ":" << prec_label(prec) << ":nrhs" << nrhs << ":" << dims[0] << "x"
    << dims[1] << "x" << dims[2] << "x" << dims[3];
  return k.str();
}

// The cache file: one JSON object whose members are
//   "<key>": {"tile_sites": N, "candidates": [n0, n1, ...], "us": [t0, t1, ...]}
// Other keys are kept as they are when the file is rewritten.
std::map<std::string, std::string> read_entries(const std::string& path) {
  std::map<std::string, std::string> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = s.find('{');
  if (i == std::string::npos) return out;
  ++i;
  for (;;) {
    const size_t q0 = s.find('"', i);
    if (q0 == std::string::npos) break;
    const size_t q1 = s.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const size_t o = s.find('{', q1);
    if (o == std::string::npos) break;
    const size_t e = s.find('}', o);
    if (e == std::string::npos) break;
    out[s.substr(q0 + 1, q1 - q0 - 1)] = s.substr(o, e - o + 1);
    i = e + 1;
  }
  return out;
}

std::vector<double> number_list(const std::string& body, const char* name) {
  std::vector<double> v;
  const size_t k = body.find(std::string("\"") + name + "\"");
  if (k == std::string::npos) return v;
  const size_t a = body.find('[', k), b = body.find(']', k);
  if (a == std::string::npos || b == std::string::npos || b < a) return v;
  std::istringstream in(body.substr(a + 1, b - a - 1));
  double x;
  char sep;
  while (in >> x) {
    v.push_back(x);
    if (!(in >> sep)) break;
  }
  return v;
}

long long number_field(const std::string& body, const char* name) {
  const size_t k = body.find(std::string("\"") + name + "\"");
  if (k == std::string::npos) return -1;
  const size_t c = body.find(':', k);
  return c == std::string::npos ? -1 : std::atoll(body.c_str() + c + 1);
}

void write_entry(const std::string& path, const std::string& key, const std::string& body) {
  auto all = read_entries(path);
  all[key] = body;
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    LQ_CHECK(f.good(), LQ_EINVAL, "cannot write the tile cache file " + path);
    f << "{\n";
    size_t n = 0;
    for (const auto& kv : all)
      f << "  \"" << kv.first << "\": " << kv.second << (++n < all.size() ? ",\n" : "\n");
    f << "}\n";
    LQ_CHECK(f.good(), LQ_EINVAL, "cannot write the tile cache file " + path);
  }
  LQ_CHECK(std::rename(tmp.c_str(), path.c_str()) == 0, LQ_EINVAL,
           "cannot replace the tile cache file " + path);
}

// Candidate tile targets: distinct tilings only (targets at or above the
// half volume all mean one tile).
std::vector<int64_t> candidates(const int dims[4], bool multi) {
  static const int64_t single[] = {4096, 16384, 65536, 262144, 1LL << 40};
  static const int64_t multi_rhs[] = {512, 1024, 2048, 8192, 32768};
  const int64_t* c = multi ? multi_rhs : single;
  std::vector<int64_t> out;
  std::vector<std::vector<int>> seen;
  for (int i = 0; i < 5; ++i) {
    int T[4];
    lq::choose_tiles(dims, c[i], T);
    std::vector<int> t(T, T + 4);
    bool dup = false;
    for (const auto& s : seen) dup = dup || s == t;
    if (dup) continue;
    seen.push_back(t);
    out.push_back(c[i]);
  }
  return out;
}

struct Scratch {  // one candidate's context and fields
  lq_ctx* ctx = nullptr;
  void *in = nullptr, *out = nullptr, *tmp = nullptr;
  ~Scratch() {
    for (void* p : {in, out, tmp})
      if (p) (void)hipFree(p);
    if (ctx) lq_destroy(ctx);
  }
};

void check(lq_ctx* ctx, lq_status st) {
  if (st != LQ_OK) throw lq::Error(st, lq_last_error(ctx));
}

// Mean time of one Schur application (reps launches after warm-ups) on a
// context whose tiles hold at most `target` sites of one parity.
double time_candidate(const int dims[4], int t_antiperiodic, int prec, int nrhs, int64_t target,
                      hipStream_t st, int T[4]) {
  const bool multi = prec == LQ_F16X;
  Scratch sc;
  if (lq_create(dims, t_antiperiodic, st, &sc.ctx) != LQ_OK)
    throw lq::Error(LQ_EINVAL, lq_last_error(nullptr));
  check(sc.ctx, multi ? lq_set_tiling(sc.ctx, 0, target) : lq_set_tiling(sc.ctx, target, 0));
  lq_ctx* ctx = sc.ctx;
  for (int k = 0; k < 4; ++k) T[k] = multi ? ctx->mr_geo.T[k] : ctx->geo.T[k];
  ctx->cur = st;
  lq::upload_unit_gauge(ctx);
  check(ctx, lq_set_clover(ctx, 0.135, 1.0));
  const size_t fb = lq_field_bytes(ctx, LQ_EVEN, prec, nrhs);
  const size_t tb = lq_field_bytes(ctx, LQ_ODD, prec, nrhs);
  LQ_CHECK(fb > 0 && tb > 0, LQ_EINVAL, "no field of this precision and nrhs");
  LQ_HIP(hipMalloc(&sc.in, fb));
  LQ_HIP(hipMalloc(&sc.out, fb));
  LQ_HIP(hipMalloc(&sc.tmp, tb));
  LQ_HIP(hipMemsetAsync(sc.in, 0, fb, st));
  constexpr int WARM = 3, REPS = 20;
  for (int r = 0; r < WARM; ++r) check(ctx, lq_schur(ctx, sc.out, sc.in, sc.tmp, 0, prec, nrhs));
  hipEvent_t e0, e1;
  LQ_HIP(hipEventCreate(&e0));
  LQ_HIP(hipEventCreate(&e1));
  float ms = 0.f;
  hipError_t err = hipEventRecord(e0, st);
  for (int r = 0; r < REPS && err == hipSuccess; ++r)
    if (lq_schur(ctx, sc.out, sc.in, sc.tmp, 0, prec, nrhs) != LQ_OK) err = hipErrorUnknown;
  if (err == hipSuccess) err = hipEventRecord(e1, st);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  LQ_HIP(err);
  return 1e3 * ms / REPS;
}

void tune(const int dims[4], int t_antiperiodic, int prec, int nrhs, const char* cache_path,
          lq_tune_report* rep) {
  const bool multi = prec == LQ_F16X;
  LQ_CHECK(dims, LQ_EINVAL, "null dims");
  LQ_CHECK(multi ? (nrhs >= 1 && nrhs <= 16)
                 : (nrhs == 1 && (prec == LQ_F64 || prec == LQ_F32 || prec == LQ_F16)),
           LQ_EINVAL, "tune LQ_F64/LQ_F32/LQ_F16 with nrhs = 1, or LQ_F16X with nrhs 1..16");
  const std::vector<int64_t> cand = candidates(dims, multi);
  LQ_CHECK((int)cand.size() <= LQ_TUNE_MAX, LQ_EINVAL, "too many candidates");
  lq_tune_report r{};
  r.ncand = (int)cand.size();
  for (int i = 0; i < r.ncand; ++i) {
    r.target[i] = cand[i];
    lq::choose_tiles(dims, cand[i], r.tiles[i]);
  }
  const std::string key = tune_key(dims, prec, nrhs);
  bool have = false;
  if (cache_path && *cache_path) {
    const auto all = read_entries(cache_path);
    const auto it = all.find(key);
    if (it != all.end()) {
      const long long best = number_field(it->second, "tile_sites");
      const std::vector<double> us = number_list(it->second, "us");
      for (int i = 0; i < r.ncand; ++i)
        if (cand[i] == best) {
          r.best = i;
          have = true;
        }
      if (have) {
        r.from_cache = 1;
        for (int i = 0; i < r.ncand && i < (int)us.size(); ++i) r.us[i] = us[i];
      }
    }
  }
  if (!have) {
    hipStream_t st = nullptr;
    LQ_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    try {
      double best = 1e300;
      for (int i = 0; i < r.ncand; ++i) {
        r.us[i] = time_candidate(dims, t_antiperiodic, prec, nrhs, cand[i], st, r.tiles[i]);
        if (r.us[i] < best) {
          best = r.us[i];
          r.best = i;
        }
      }
    } catch (...) {
      (void)hipStreamDestroy(st);
      throw;
    }
    LQ_HIP(hipStreamDestroy(st));
    if (cache_path && *cache_path) {
      std::ostringstream b;
      b << "{\"tile_sites\": " << cand[r.best] << ", \"candidates\": [";
      for (int i = 0; i < r.ncand; ++i) b << (i ? ", " : "") << cand[i];
      b << "], \"us\": [";
      for (int i = 0; i < r.ncand; ++i) b << (i ? ", " : "") << r.us[i];
      b << "]}";
      write_entry(cache_path, key, b.str());
    }
  }
  if (rep) *rep = r;
}

}  // namespace

extern "C" {

lq_status lq_set_tiling(lq_ctx* ctx, int64_t tile_sites, int64_t mr_tile_sites) {
  if (!ctx) return LQ_EINVAL;
  try {
    LQ_CHECK(tile_sites == 0 || tile_sites >= 64, LQ_EINVAL, "tile_sites: 0 or at least 64");
    LQ_CHECK(mr_tile_sites == 0 || mr_tile_sites >= 64, LQ_EINVAL,
             "mr_tile_sites: 0 or at least 64");
    LQ_CHECK(!ctx->have_gauge && !ctx->work && !ctx->mrwork && !ctx->mr_nbr && !ctx->sap &&
                 !ctx->kwork && !ctx->bwork,
             LQ_ESTATE, "the tiling is fixed once a gauge field or work space exists");
    if (tile_sites > 0) {
      lq::choose_tiles(ctx->geo.L, tile_sites, ctx->geo.T);
      lq::geo_finish(ctx->geo);
    }
    if (mr_tile_sites > 0) {
      lq::choose_tiles(ctx->mr_geo.L, mr_tile_sites, ctx->mr_geo.T);
      lq::geo_finish(ctx->mr_geo);
    }
    return LQ_OK;
  } catch (const lq::Error& e) {
    ctx->err = e.what();
    return e.code;
  }
}

lq_status lq_get_tiling(const lq_ctx* ctx, int tiles[4], int mr_tiles[4]) {
  if (!ctx) return LQ_EINVAL;
  for (int k = 0; k < 4; ++k) {
    if (tiles) tiles[k] = ctx->geo.T[k];
    if (mr_tiles) mr_tiles[k] = ctx->mr_geo.T[k];
  }
  return LQ_OK;
}

lq_status lq_tune_tiles(const int dims[4], int t_antiperiodic, int prec, int nrhs,
                        const char* cache_path, lq_tune_report* rep) {
  try {
    tune(dims, t_antiperiodic, prec, nrhs, cache_path, rep);
    g_tune_error.clear();
    return LQ_OK;
  } catch (const lq::Error& e) {
    g_tune_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_tune_error = e.what();
    return LQ_EINVAL;
  }
}

const char* lq_tune_last_error(void) { return g_tune_error.c_str(); }

}  // extern "C"
