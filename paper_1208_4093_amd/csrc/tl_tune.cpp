// Autotuned launch choices: the set edge of the partition into sets (section
// 2.2), the overlap of the relaxation region (section 2.2 end) and the
// relaxation sweeps per set (the inner solve of Eq. 12), measured per lattice
// shape and precision and kept in a process-wide table that a text file
// (TL_TUNE_CACHE) persists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "tl.h"
#include "tl_runtime.h"

namespace tl {
namespace {

struct TuneKey {
  int bx, by, mixed;
  bool operator<(const TuneKey& o) const {
    return std::tie(bx, by, mixed) < std::tie(o.bx, o.by, o.mixed);
  }
};

int side_bucket(int s) { return (int)std::lround(2.0 * std::log2((double)std::max(s, 1))); }

TuneKey key_of(int nx, int ny, bool mixed) { return {side_bucket(nx), side_bucket(ny), mixed ? 1 : 0}; }

bool valid_entry(const tl_tune_entry& e) {
  return (e.set_edge == 16 || e.set_edge == 32 || e.set_edge == 64) &&
         (e.overlap == -1 || e.overlap == 1 || e.overlap == 2 || e.overlap == 4) &&
         e.inner_iters >= 1 && e.inner_iters <= 1024 && e.nx >= 2 && e.ny >= 2;
}

constexpr const char* kHeader = "# tl tuning table v1: bx by mixed set_edge overlap inner_iters nx ny ms";

class TuneTable {
 public:
  // Entry for a key; loads TL_TUNE_CACHE on the table's first use.
  bool find(const TuneKey& k, tl_tune_entry* out) {
    std::lock_guard<std::mutex> l(mu_);
    load_env_locked();
    auto it = m_.find(k);
    if (it == m_.end()) return false;
    *out = it->second;
    return true;
  }
  void put(const TuneKey& k, const tl_tune_entry& e) {
    std::lock_guard<std::mutex> l(mu_);
    load_env_locked();
    m_[k] = e;
    const char* path = getenv("TL_TUNE_CACHE");
    if (path && *path) (void)save_locked(path);
  }
  tl_status load(const char* path) {
    std::lock_guard<std::mutex> l(mu_);
    load_env_locked();
    std::map<TuneKey, tl_tune_entry> add;
    const tl_status s = parse(path, &add);
    if (s != TL_OK) return s;
    for (auto& kv : add) m_[kv.first] = kv.second;
    return TL_OK;
  }
  tl_status save(const char* path) {
    std::lock_guard<std::mutex> l(mu_);
    load_env_locked();
    return save_locked(path);
  }
  void clear() {
    std::lock_guard<std::mutex> l(mu_);
    env_loaded_ = true;
    m_.clear();
  }

 private:
  void load_env_locked() {
    if (env_loaded_) return;
    env_loaded_ = true;
    const char* path = getenv("TL_TUNE_CACHE");
    if (!path || !*path) return;
    std::map<TuneKey, tl_tune_entry> add;
    if (parse(path, &add) == TL_OK) m_ = add;   // a missing or malformed file: empty table
  }
  static tl_status parse(const char* path, std::map<TuneKey, tl_tune_entry>* out) {
    FILE* f = fopen(path, "r");
    if (!f) return TL_E_INVAL;
    char line[512];
    tl_status s = TL_OK;
    while (fgets(line, sizeof line, f)) {
      const char* c = line;
      while (*c == ' ' || *c == '\t') ++c;
      if (*c == '#' || *c == '\n' || *c == '\0') continue;
      TuneKey k{};
      tl_tune_entry e{};
      char tail[8];
      const int got = sscanf(c, "%d %d %d %d %d %d %d %d %lf %7s", &k.bx, &k.by, &k.mixed,
                             &e.set_edge, &e.overlap, &e.inner_iters, &e.nx, &e.ny, &e.ms, tail);
      if (got != 9 || (k.mixed != 0 && k.mixed != 1) || !valid_entry(e) ||
          key_of(e.nx, e.ny, k.mixed != 0).bx != k.bx || key_of(e.nx, e.ny, k.mixed != 0).by != k.by) {
        s = TL_E_INVAL;
        break;
      }
      (*out)[k] = e;
    }
    fclose(f);
    if (s != TL_OK) out->clear();
    return s;
  }
  tl_status save_locked(const char* path) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return TL_E_INVAL;
    fprintf(f, "%s\n", kHeader);
    for (auto& kv : m_) {
      const tl_tune_entry& e = kv.second;
      fprintf(f, "%d %d %d %d %d %d %d %d %.17g\n", kv.first.bx, kv.first.by, kv.first.mixed,
              e.set_edge, e.overlap, e.inner_iters, e.nx, e.ny, e.ms);
    }
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path) != 0) return TL_E_INVAL;
    return TL_OK;
  }

  std::mutex mu_;
  std::map<TuneKey, tl_tune_entry> m_;
  bool env_loaded_ = false;
};

TuneTable& table() {
  static TuneTable t;
  return t;
}

}  // namespace

int tuned_set_edge(int nx, int ny) {
  tl_tune_entry e;
  if (table().find(key_of(nx, ny, true), &e) || table().find(key_of(nx, ny, false), &e))
    return e.set_edge;
  return 0;
}

void apply_tuned(const tl_lattice* L, Opts* o) {
  if (!o->overlap_default && !o->inner_default) return;
  tl_tune_entry e;
  if (!table().find(key_of(L->g.nx, L->g.ny, o->mixed), &e) || e.set_edge != L->g.E) return;
  if (o->overlap_default) o->overlap = e.overlap < 0 ? 0 : e.overlap;
  if (o->inner_default) o->inner = e.inner_iters;
}

}  // namespace tl

using namespace tl;

extern "C" {

tl_status tl_tune(const tl_lattice_desc* desc, const double* f_dev, const tl_opts* opts,
                  tl_tune_entry* out, void* hip_stream) {
  if (!desc || !f_dev || !out || desc->nx < 2 || desc->ny < 2) return TL_E_INVAL;
  Opts probe;
  if (resolve_opts(opts, &probe) != TL_OK || probe.trace || probe.profile) return TL_E_INVAL;
  const bool mixed = probe.mixed;
  const int nx = desc->nx, ny = desc->ny;
  double* u = nullptr;
  if (hipMalloc((void**)&u, (size_t)nx * ny * 2 * sizeof(double)) != hipSuccess) return TL_E_NOMEM;
  tl_opts base = opts ? *opts : tl_opts{};
  base.trace = nullptr;
  base.profile = 0;
  base.warm_start = 0;

  struct Cand { int E, ov, inner; };
  std::map<int, tl_lattice*> lats;   // by set edge
  tl_status err = TL_OK;
  auto lattice_for = [&](int E) -> tl_lattice* {
    auto it = lats.find(E);
    if (it != lats.end()) return it->second;
    tl_lattice_desc d = *desc;
    d.set_edge = E;
    tl_lattice* L = nullptr;
    const tl_status s = tl_lattice_create(&d, hip_stream, &L);
    if (s != TL_OK) { err = s; L = nullptr; }
    lats[E] = L;
    return L;
  };
  // one candidate: a warm-up solve (work space allocation, coarse space),
  // then two timed solves; +inf when any of them fails to converge
  auto measure = [&](const Cand& c) -> double {
    tl_lattice* L = lattice_for(c.E);
    if (!L) return INFINITY;
    tl_opts o = base;
    o.overlap = c.ov;
    o.inner_iters = c.inner;
    double best = INFINITY;
    for (int rep = 0; rep < 3; ++rep) {
      tl_info info{};
      const auto t0 = std::chrono::steady_clock::now();
      const tl_status s = tl_solve(L, f_dev, u, &o, &info, hip_stream);
      const auto t1 = std::chrono::steady_clock::now();
      if (s != TL_OK) return INFINITY;
      if (rep > 0) best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    return best;
  };

  const int side = std::max(nx, ny);
  std::vector<int> edges;
  for (int E : {16, 32, 64})
    if (E <= side) edges.push_back(E);
  if (edges.empty()) edges.push_back(16);
  int E0 = default_set_edge(nx, ny);
  if (std::find(edges.begin(), edges.end(), E0) == edges.end()) E0 = edges.front();
  Cand best{E0, 2, default_inner_iters(E0, mixed)};
  double best_ms = INFINITY;
  std::map<std::tuple<int, int, int>, double> seen;
  auto consider = [&](const Cand& c) {
    const auto key = std::make_tuple(c.E, c.ov, c.inner);
    auto it = seen.find(key);
    const double ms = it != seen.end() ? it->second : (seen[key] = measure(c));
    if (ms < best_ms) { best_ms = ms; best = c; }
  };
  // set edge (its own default sweeps), then overlap, then sweeps
  for (int E : edges) consider({E, 2, default_inner_iters(E, mixed)});
  const int Eb = best.E;
  for (int ov : {1, 2, 4}) consider({Eb, ov, best.inner});
  const int ovb = best.ov, ib = best.inner;
  for (int d : {-8, -4, 4, 8})
    if (ib + d >= 4) consider({Eb, ovb, ib + d});

  for (auto& kv : lats)
    if (kv.second) tl_lattice_destroy(kv.second);
  (void)hipFree(u);
  if (!std::isfinite(best_ms)) return err != TL_OK ? err : TL_E_NOCONV;
  tl_tune_entry e{};
  e.set_edge = best.E;
  e.overlap = best.ov <= 0 ? -1 : best.ov;
  e.inner_iters = best.inner;
  e.nx = nx;
  e.ny = ny;
  e.ms = best_ms;
  table().put(key_of(nx, ny, mixed), e);
  *out = e;
  return TL_OK;
}

tl_status tl_tune_lookup(int32_t nx, int32_t ny, tl_precision precision, tl_tune_entry* out) {
  if (!out || nx < 2 || ny < 2) return TL_E_INVAL;
  *out = tl_tune_entry{};
  (void)table().find(key_of(nx, ny, precision == TL_MIXED), out);
  return TL_OK;
}

tl_status tl_tune_load(const char* path) { return path ? table().load(path) : TL_E_INVAL; }

tl_status tl_tune_save(const char* path) { return path ? table().save(path) : TL_E_INVAL; }

tl_status tl_tune_clear(void) {
  table().clear();
  return TL_OK;
}

}  // extern "C"
