// Host runtime of the hierarchical lattice solver: the C ABI of include/tl.h.
//
// A solve enqueues, per outer iteration, the tile kernel (update, residual,
// relaxation, set rows of the upper-level system), the boundary-block kernel
// and the persistent upper-level kernel, which also evaluates the stop test
// and raises a device flag.  The host only reads that flag between chunks of
// iterations; kernels enqueued after the flag is raised return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "tl.h"
#include "tl_internal.h"
#include "tl_runtime.h"

namespace tl {

namespace {

tl_status from_hip(hipError_t e) {
  if (e == hipSuccess) return TL_OK;
  if (e == hipErrorOutOfMemory) return TL_E_NOMEM;
  return TL_E_DEVICE;
}

#define TL_TRY(expr)                         \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return from_hip(e_); \
  } while (0)

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v && *v ? std::atoi(v) : dflt;
}

}  // namespace

int default_set_edge(int nx, int ny) {
  const int side = std::max(nx, ny);
  if (side <= 160) return 16;
  if (side <= 2048) return 32;
  return 64;
}

Geo make_geo(int nx, int ny, int E) {
  Geo g;
  g.nx = nx;
  g.ny = ny;
  g.pitch = ((nx + LPAD + 1 + 31) / 32) * 32;
  g.E = E;
  g.mx = (nx + E - 1) / E;
  g.my = (ny + E - 1) / E;
  g.M = g.mx * g.my;
  return g;
}

size_t padded_nodes(const Geo& g) { return (size_t)(g.ny + 2) * g.pitch; }

size_t work_bytes(const Geo& g, bool mixed, int hist_cap) {
  const size_t np = padded_nodes(g), M = g.M;
  size_t b = 2 * np * sizeof(double2) + 2 * np * (mixed ? sizeof(float2) : sizeof(double2));
  b += M * (Q + KROW + Q + NRM + NDIR * Q * Q + 2 * Q * Q + 11 * Q) * sizeof(double);
  b += 2 * COARSE_MAX_WG * REDW * sizeof(double) + (size_t)hist_cap * sizeof(double);
  b += COARSE_MAX_WG * sizeof(unsigned);
  b += sizeof(Ctrl);
  return b;
}

void Work::release() {
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  events.clear();
  for (void* p : allocs) (void)hipFree(p);
  allocs.clear();
  if (ctrl_host) (void)hipHostFree(ctrl_host);
  ctrl_host = nullptr;
}

tl_status Work::alloc(const Geo& g_, bool mixed_, int hist_cap_) {
  g = g_;
  mixed = mixed_;
  hist_cap = hist_cap_;
  const size_t np = padded_nodes(g), M = g.M;
  auto get = [&](size_t bytes, void** p) -> hipError_t {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return e;
    allocs.push_back(*p);
    return hipMemset(*p, 0, bytes);
  };
  void* p;
  for (int k = 0; k < 2; ++k) {
    TL_TRY(get(np * sizeof(double2), &p)); u[k] = (double2*)p;
    TL_TRY(get(np * (mixed ? sizeof(float2) : sizeof(double2)), &p)); d[k] = p;
  }
  TL_TRY(get(M * Q * sizeof(double), &p)); a = (double*)p;
  TL_TRY(get(M * KROW * sizeof(double), &p)); krow = (double*)p;
  TL_TRY(get(M * Q * sizeof(double), &p)); force = (double*)p;
  TL_TRY(get(M * NRM * sizeof(double), &p)); nrm = (double*)p;
  TL_TRY(get(M * NDIR * Q * Q * sizeof(double), &p)); off = (double*)p;
  TL_TRY(get(M * Q * Q * sizeof(double), &p)); bdiag = (double*)p;
  TL_TRY(get(M * Q * Q * sizeof(double), &p)); binv = (double*)p;
  double** vecs[] = {&cr, &cu, &cw, &cz, &cq, &cs, &cp, &cn, &pub0, &pub1, &pub2};
  for (double** v : vecs) {
    TL_TRY(get(M * Q * sizeof(double), &p));
    *v = (double*)p;
  }
  TL_TRY(get(2 * COARSE_MAX_WG * REDW * sizeof(double), &p)); red = (double*)p;
  TL_TRY(get((size_t)hist_cap * sizeof(double), &p)); hist = (double*)p;
  TL_TRY(get(sizeof(Ctrl), &p)); ctrl = (Ctrl*)p;
  TL_TRY(get(COARSE_MAX_WG * sizeof(unsigned), &p)); flags = (unsigned*)p;
  TL_TRY(hipHostMalloc((void**)&ctrl_host, sizeof(Ctrl), hipHostMallocDefault));
  bytes = work_bytes(g, mixed, hist_cap);
  return TL_OK;
}

// Launch shape of the upper-level kernel: about `per` sets per workgroup, at
// most one workgroup per CU and few enough that each one's LDS windows fit;
// the own vectors and blocks go to LDS when there is room.
constexpr size_t kCoarseLdsCap = COARSE_DYN_LDS_MAX;

CoarseShape coarse_shape(const Geo& g) {
  const int per = std::max(1, env_int("TL_COARSE_SETS_PER_WG", 16));
  CoarseShape c;
  c.nwg = std::max(1, std::min((g.M + per - 1) / per, COARSE_MAX_WG));
  while (c.nwg < COARSE_MAX_WG && coarse_lds_bytes(g, c.nwg, 0, 0, 0) > kCoarseLdsCap) ++c.nwg;
  c.two_level = coarse_lds_bytes(g, c.nwg, 0, 0, 1) <= kCoarseLdsCap;
  c.vec_lds = coarse_lds_bytes(g, c.nwg, 1, 0, c.two_level) <= kCoarseLdsCap;
  c.blk_lds = c.vec_lds && coarse_lds_bytes(g, c.nwg, 1, 1, c.two_level) <= kCoarseLdsCap;
  if (env_int("TL_COARSE_NO_LDS", 0)) c.vec_lds = c.blk_lds = 0;
  return c;
}

// Relaxation sweeps per set when the caller leaves the field at 0.  Measured
// with the two-level upper level (1024^2 and 2048^2 with 32 x 32 sets,
// 4096^2 with 64 x 64): solve time falls from 10 sweeps up to about 16 for
// 32 x 32 sets (1024^2 float64 70 -> 65 ms) and about 24 for 64 x 64
// (4096^2 mixed 1148 -> 911 ms), then rises again.  Since the float64 tile
// of a 32 x 32 set runs two to a CU its sweeps are cheaper and 20 is best
// in that form (1024^2 42.5 -> 40.5 ms, 2048^2 lognormal 117.8 -> 112.9 ms,
// 512^2 26.0 -> 23.5 ms; 18, 22 and 24 are slower); the float32 form stays
// fastest at 16.
int default_inner_iters(int E, bool mixed) { return E >= 64 ? 24 : (E == 32 && !mixed ? 20 : 16); }

// Defaults when the caller leaves a field at 0.  Measured on 1024^2 (unit EA,
// 32 x 32 sets), 2048^2 and 4096^2 (lognormal EA, 32 and 64 sets) to 1e-8:
// widening each relaxation region by 2 nodes cuts the outer iterations 2-3x
// for 1.3-1.9x more tile time, and capping the upper-level PCG at 100
// iterations (relative tolerance 0.1) avoids long solves whose extra
// accuracy the outer iteration does not use; together about 2x faster.
constexpr int kDefaultOverlap = 2;

// The upper-level PCG's cap and relative tolerance when the caller leaves them
// at 0, measured to 1e-8 (1e-10 at 16384^2):
//  - from 16384 sets on (8192^2 and 16384^2 with 64 x 64 sets) a tighter
//    upper-level solve, 0.05 with a cap of 200, cuts the outer iterations
//    enough to pay for itself (16384^2: 434 -> 362 outer iterations, 16.4 ->
//    14.4 s; 8192^2: 3.34 -> 3.24 s);
//  - below that the float64 form with sets of at most 32 x 32 does better
//    with a looser one, 0.15 (512^2 to 3000^2: 1-7 % faster), while with
//    64 x 64 sets, and in the mixed form, 0.15 costs outer iterations
//    (4096^2 float64 +4 %, 2048^2 mixed +27 %) and 0.1 stays;
//  - lattices of at most 256 sets (sides up to 512 with 32 x 32 sets) stop
//    the upper-level PCG after 20 iterations in float64 and 25 in the mixed
//    form.  Fused with others, a lattice's long upper-level solve holds the
//    whole launch; capped, the 256-lattice batch of sides 32-512 runs 6 %
//    (float64) and 3 % (mixed) faster on three seed sets of its lattices,
//    with the same outer iterations to within a few.  At 1024 sets (1024^2)
//    a cap of 20 costs outer iterations (float64 104 -> 172), so larger
//    lattices keep 100.
constexpr int kLargeUpperLevel = 16384;
constexpr int kSmallUpperLevel = 256;
int default_coarse_iters(int M, bool mixed) {
  if (M >= kLargeUpperLevel) return 200;
  if (M <= kSmallUpperLevel) return mixed ? 25 : 20;
  return 100;
}
double default_coarse_rtol(int M, int E, bool mixed) {
  if (M >= kLargeUpperLevel) return 0.05;
  return !mixed && E <= 32 ? 0.15 : 0.1;
}

tl_status resolve_opts(const tl_opts* o, Opts* r) {
  r->mixed = o && o->precision == TL_MIXED;
  r->rtol = o && o->rtol > 0.0 ? o->rtol : 1e-8;
  r->max_iters = o && o->max_iters > 0 ? o->max_iters : 20000;
  r->inner = o && o->inner_iters > 0 ? o->inner_iters : 0;   // 0: by set edge, below
  r->overlap = !o || o->overlap == 0 ? kDefaultOverlap : (o->overlap < 0 ? 0 : o->overlap);
  r->coarse_iters = o && o->coarse_iters > 0 ? o->coarse_iters : 0;   // 0: by lattice size, below
  r->coarse_rtol = o && o->coarse_rtol > 0.0 ? o->coarse_rtol : 0.0;
  r->warm = o ? o->warm_start : 0;
  r->trace = o ? o->trace : nullptr;
  r->profile = o ? o->profile : 0;
  r->exact = o && o->local_solve == 1;
  r->overlap_default = !o || o->overlap == 0;
  r->inner_default = !o || o->inner_iters == 0;
  if (!(r->rtol > 0.0) || r->max_iters < 0 || r->inner < 0 || !tile_overlap_supported(r->overlap))
    return TL_E_INVAL;
  if (o && (o->local_solve < 0 || o->local_solve > 1)) return TL_E_INVAL;
  if (r->exact && r->mixed) return TL_E_INVAL;
  return TL_OK;
}

// Arguments of one outer iteration's kernels for one solve (fixed for the
// whole solve: the iteration counter and stop flag live in the control block).
void make_iteration_args(const tl_lattice* L, Work* w, const Opts& o, const double* f,
                         TileArgs* ta, OffArgs* oa, BlockArgs* ba, CoarseArgs* ca) {
  ta->u0 = w->u[0];
  ta->u1 = w->u[1];
  ta->d0 = w->d[0];
  ta->d1 = w->d[1];
  ta->a = w->a;
  ta->f = (const double2*)f;
  ta->krow = w->krow;
  ta->force = w->force;
  ta->nrm = w->nrm;
  ta->ctrl = w->ctrl;
  ta->inner_iters = o.inner > 0 ? o.inner : default_inner_iters(L->g.E, o.mixed);
  ta->rhs_mode = L->ufix != nullptr;
  {
    const int R = L->g.E + 2 * o.overlap;
    const int bi = o.overlap == 4 ? 3 : o.overlap;
    ta->band = o.exact ? L->band[bi] : nullptr;
    ta->band_stride = band_set_doubles(R);
    ta->band_bs = band_bs(R);
  }
  oa->d0 = w->d[0];
  oa->d1 = w->d[1];
  oa->off = w->off;
  oa->ctrl = w->ctrl;
  ba->g1 = L->g1;
  ba->krow = w->krow;
  ba->bdiag = w->bdiag;
  ba->binv = w->binv;
  ba->ctrl = w->ctrl;
  ca->g1 = L->g1;
  ca->krow = w->krow;
  ca->force = w->force;
  ca->nrm = w->nrm;
  ca->off = w->off;
  ca->bdiag = w->bdiag;
  ca->binv = w->binv;
  ca->a = w->a;
  ca->cr = w->cr;
  ca->cu = w->cu;
  ca->cw = w->cw;
  ca->cz = w->cz;
  ca->cq = w->cq;
  ca->cs = w->cs;
  ca->cp = w->cp;
  ca->cn = w->cn;
  ca->pub0 = w->pub0;
  ca->pub1 = w->pub1;
  ca->pub2 = w->pub2;
  ca->red = w->red;
  ca->flags = w->flags;
  ca->hist = (o.trace && o.trace->residual_history) ? o.trace->residual_history : w->hist;
  ca->tr_kdiag = o.trace ? o.trace->kdiag : nullptr;
  ca->tr_koff = o.trace ? o.trace->koff : nullptr;
  ca->tr_force = o.trace ? o.trace->force : nullptr;
  ca->tr_coef = o.trace ? o.trace->coef : nullptr;
  ca->ctrl = w->ctrl;
  ca->max_iters = o.max_iters;
  ca->coarse_iters = o.coarse_iters > 0 ? o.coarse_iters : default_coarse_iters(L->g.M, o.mixed);
  ca->coarse_rtol = o.coarse_rtol > 0.0 ? o.coarse_rtol : default_coarse_rtol(L->g.M, L->g.E, o.mixed);
  ca->rtol = o.rtol;
  ca->warm = env_int("TL_COARSE_WARM", 1);
  ca->coarse_ref = env_int("TL_COARSE_REF", 0);
  ca->spin_limit = 1u << 22;
  const CoarseShape cs = coarse_shape(L->g);
  ca->nwg = cs.nwg;
  ca->vec_lds = cs.vec_lds;
  ca->blk_lds = cs.blk_lds;
  // the coarse space, when built and laid out for this workgroup count
  const bool two = L->agg_ready && L->naggr > 0 && cs.two_level && L->agg_nwg == cs.nwg &&
                   env_int("TL_COARSE_2LEVEL", 1) != 0;
  ca->agg_inv = two ? L->agg_inv : nullptr;
  ca->agg_xy = two ? L->agg_xy : nullptr;
  ca->naggr = two ? L->naggr : 0;
  ca->agg_sets = two ? L->agg_sets : 1;
  ca->agg_g = two ? L->agg_g : 1;
}

tl_status ensure_coarse_space(tl_lattice* L, Work* w, const Opts& o, const double* f,
                              hipStream_t st) {
  if (L->agg_ready || L->naggr == 0 || env_int("TL_COARSE_2LEVEL", 1) == 0) return TL_OK;
  std::lock_guard<std::mutex> lock(L->agg_mu);
  if (L->agg_ready) return TL_OK;
  // the boundary blocks of the just-initialised state (relaxation increments
  // zero) carry the constant mode 1-6 corners that the coarse space needs
  TileArgs ta;
  OffArgs oa;
  BlockArgs ba;
  CoarseArgs ca;
  make_iteration_args(L, w, o, f, &ta, &oa, &ba, &ca);
  TL_TRY(launch_offdiag(o.mixed, L->g, L->ea, L->mask, oa, st));
  TL_TRY(launch_agg_setup(L->g, L->g1, w->off, L->agg_xy, L->agg_sets, L->naggr, L->agg_inv, st));
  TL_TRY(hipStreamSynchronize(st));
  L->agg_ready = true;
  return TL_OK;
}

tl_status ensure_band(tl_lattice* L, const Opts& o, hipStream_t st) {
  if (!o.exact) return TL_OK;
  if (o.mixed || L->g.E > 32) return TL_E_INVAL;
  const int bi = o.overlap == 4 ? 3 : o.overlap;
  std::lock_guard<std::mutex> lock(L->band_mu);
  if (L->band[bi]) return TL_OK;
  const int R = L->g.E + 2 * o.overlap;
  void* p = nullptr;
  const size_t bytes = band_set_doubles(R) * sizeof(double) * (size_t)L->g.M;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return TL_E_NOMEM;
  }
  hipError_t e = launch_band_factor(L->g, o.overlap, L->ea, L->mask, (double*)p, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return from_hip(e);
  }
  L->allocs.push_back(p);
  L->bytes += bytes;
  L->band[bi] = (double*)p;
  return TL_OK;
}

// Enqueue one outer iteration of one solve (ev: optional 4 timing events).
tl_status enqueue_iteration(const tl_lattice* L, Work* w, const Opts& o, const double* f,
                            hipStream_t st, hipEvent_t* ev) {
  TileArgs ta;
  OffArgs oa;
  BlockArgs ba;
  CoarseArgs ca;
  make_iteration_args(L, w, o, f, &ta, &oa, &ba, &ca);
  if (ev) TL_TRY(hipEventRecord(ev[0], st));
  TL_TRY(launch_tile(o.mixed, o.overlap, L->g, L->ea, L->mask, ta, st));
  if (ev) TL_TRY(hipEventRecord(ev[1], st));
  TL_TRY(launch_offdiag(o.mixed, L->g, L->ea, L->mask, oa, st));
  TL_TRY(launch_blockinv(L->g, ba, st));
  if (ev) TL_TRY(hipEventRecord(ev[2], st));
  TL_TRY(launch_coarse(L->g, ca, st));
  if (ev) TL_TRY(hipEventRecord(ev[3], st));
  return TL_OK;
}

tl_status certify(const tl_lattice* L, const double* f, const double* u, double* r,
                  double out3[3], hipStream_t st) {
  TL_TRY(launch_residual(L->g, L->ea, L->mask, (const double2*)f, (const double2*)u, L->ufix,
                         (double2*)r, L->res_part, L->res_out, st));
  TL_TRY(hipMemcpyAsync(L->out5_host, L->res_out, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
  TL_TRY(hipStreamSynchronize(st));
  const double* o5 = L->out5_host;
  out3[0] = o5[2] > 0.0 ? o5[0] / o5[2] : o5[0];
  out3[1] = o5[3] > 0.0 ? std::sqrt(o5[1] / o5[3]) : std::sqrt(o5[1]);
  out3[2] = o5[4];
  return TL_OK;
}

tl_status run_solve(tl_lattice* L, Work* w, const Opts& o, const double* f, double* u,
                    tl_info* info, hipStream_t st, Ctrl* ctrl_host, bool use_events) {
  using Clock = std::chrono::steady_clock;
  const auto t_start = Clock::now();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto drop_events = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    e0 = e1 = nullptr;
  };
  if (use_events) {
    TL_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { drop_events(); return TL_E_DEVICE; }
  }
  hipError_t he = launch_init_state(L->g, L->mask, L->ufix, (const double2*)u, o.warm, w->u[0],
                                    w->u[1], w->d[0], w->d[1], o.mixed, w->a, w->flags, w->ctrl, st);
  if (he != hipSuccess) { drop_events(); return from_hip(he); }
  {
    const tl_status cs = ensure_coarse_space(L, w, o, f, st);
    if (cs != TL_OK) { drop_events(); return cs; }
  }
  if (e0 && (he = hipEventRecord(e0, st)) != hipSuccess) { drop_events(); return from_hip(he); }
  const int nwg = coarse_shape(L->g).nwg;
  int k = 0, chunk = 4;
  tl_status st_run = TL_OK;
  double t_tile = 0.0, t_off = 0.0, t_coarse = 0.0;
  int n_timed = 0;
  const bool profile = use_events && o.profile;
  for (;;) {
    const int k0 = k;
    if (profile) {
      while ((int)w->events.size() < 4 * chunk) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { st_run = TL_E_DEVICE; break; }
        w->events.push_back(e);
      }
      if (st_run != TL_OK) break;
    }
    {
      // the chunk's persistent upper-level grids are admitted process-wide
      // and the guard waits for the chunk before it is released
      PersistentGuard guard(nwg, st);
      for (int c = 0; c < chunk && k <= o.max_iters; ++c, ++k) {
        // profile = N > 1 times every N-th iteration (each event record adds a
        // few microseconds between kernels)
        const bool timed = profile && k % std::max(o.profile, 1) == 0;
        st_run = enqueue_iteration(L, w, o, f, st, timed ? &w->events[4 * c] : nullptr);
        if (st_run != TL_OK) break;
      }
      if (st_run == TL_OK &&
          hipMemcpyAsync(ctrl_host, w->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st) != hipSuccess)
        st_run = TL_E_DEVICE;
      if (st_run == TL_OK && hipStreamSynchronize(st) != hipSuccess) st_run = TL_E_DEVICE;
    }
    if (st_run != TL_OK) break;
    if (profile) {
      // iterations after the one that stopped the solve are no-ops: not counted
      const int last = ctrl_host->done ? ctrl_host->iters : k - 1;
      for (int kk = k0; kk <= std::min(last, k - 1); ++kk) {
        if (kk % std::max(o.profile, 1) != 0) continue;
        hipEvent_t* ev = &w->events[4 * (kk - k0)];
        float a = 0.f, b = 0.f, c = 0.f;
        if (hipEventElapsedTime(&a, ev[0], ev[1]) != hipSuccess ||
            hipEventElapsedTime(&b, ev[1], ev[2]) != hipSuccess ||
            hipEventElapsedTime(&c, ev[2], ev[3]) != hipSuccess) {
          st_run = TL_E_DEVICE;
          break;
        }
        t_tile += a;
        t_off += b;
        t_coarse += c;
        ++n_timed;
      }
      if (st_run != TL_OK) break;
    }
    if (ctrl_host->err) { st_run = TL_E_DEVICE; break; }
    if (ctrl_host->done) break;
    if (k > o.max_iters) { st_run = TL_E_DEVICE; break; }
    chunk = std::min(chunk * 2, 64);
  }
  if (st_run != TL_OK) {
    (void)hipStreamSynchronize(st);
    drop_events();
    return st_run;
  }
  const Ctrl c = *ctrl_host;
  const int kf = c.iters;
  if (e1 && (he = hipEventRecord(e1, st)) != hipSuccess) { drop_events(); return from_hip(he); }
  he = launch_copy_out(L->g, w->u[(kf + 1) & 1], (double2*)u, st);
  if (he == hipSuccess && o.trace && o.trace->delta && kf >= 1)
    he = launch_copy_delta(o.mixed, L->g, w->d[kf & 1], (double2*)o.trace->delta, st);
  float ms = 0.f;
  if (he == hipSuccess && e1) he = hipEventSynchronize(e1);
  if (he == hipSuccess && e1) he = hipEventElapsedTime(&ms, e0, e1);
  drop_events();
  if (he != hipSuccess) return from_hip(he);
  double out3[3];
  tl_status cs = certify(L, f, u, nullptr, out3, st);
  if (cs != TL_OK) return cs;
  if (!use_events) ms = (float)std::chrono::duration<double, std::milli>(Clock::now() - t_start).count();
  if (info) {
    info->status = (tl_status)c.status;
    info->iters = kf;
    info->rel_res_l1 = out3[0];
    info->rel_res_l2 = out3[1];
    info->energy = out3[2];
    info->ms = ms;
    info->coarse_iters = c.coarse_iters;
    info->tile_ms = t_tile;
    info->offdiag_ms = t_off;
    info->coarse_ms = t_coarse;
    info->tile_launches = n_timed;
  }
  if (c.status == 0 && !(std::isfinite(out3[0]) && std::isfinite(out3[1]))) return TL_E_NONFINITE;
  return (tl_status)c.status;
}

// ---------------------------------------------------------------------------
// Admission of persistent upper-level grids (see PersistentGuard).
// ---------------------------------------------------------------------------
namespace {

constexpr int kXcds = 8;          // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kMaxDevices = 64;

struct DeviceGate {
  std::mutex mu;
  std::condition_variable cv;
  int cap = 0;                    // CUs per XCD
  int used = 0;                   // CUs per XCD claimed by the grids in flight
  int in_flight = 0;
};
DeviceGate g_gates[kMaxDevices];

}  // namespace

PersistentGuard::PersistentGuard(int nwg, hipStream_t stream) : stream_(stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
  DeviceGate& G = g_gates[dev];
  std::unique_lock<std::mutex> lock(G.mu);
  if (G.cap == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
    G.cap = std::max(1, cus / kXcds);
  }
  const int demand = (std::max(nwg, 1) + kXcds - 1) / kXcds;
  G.cv.wait(lock, [&] { return G.in_flight == 0 || G.used + demand <= G.cap; });
  G.used += demand;
  ++G.in_flight;
  dev_ = dev;
  demand_ = demand;
}

PersistentGuard::~PersistentGuard() {
  (void)hipStreamSynchronize(stream_);
  DeviceGate& G = g_gates[dev_];
  {
    std::lock_guard<std::mutex> lock(G.mu);
    G.used -= demand_;
    --G.in_flight;
  }
  G.cv.notify_all();
}

Work* lattice_work(tl_lattice* L, bool mixed, int hist_cap, tl_status* err) {
  Work*& w = L->work[mixed ? 1 : 0];
  if (w && w->hist_cap >= hist_cap) return w;
  if (w) {
    w->release();
    delete w;
    w = nullptr;
  }
  w = new (std::nothrow) Work();
  if (!w) { *err = TL_E_NOMEM; return nullptr; }
  tl_status s = w->alloc(L->g, mixed, hist_cap);
  if (s != TL_OK) {
    w->release();
    delete w;
    w = nullptr;
    *err = s;
    return nullptr;
  }
  return w;
}

}  // namespace tl

using namespace tl;

extern "C" {

const char* tl_strerror(tl_status s) {
  switch (s) {
    case TL_OK: return "ok";
    case TL_PENDING: return "pending";
    case TL_E_INVAL: return "invalid argument";
    case TL_E_NOMEM: return "device out of memory";
    case TL_E_NOCONV: return "not converged within max_iters";
    case TL_E_DEVICE: return "HIP runtime or device error";
    case TL_E_BUDGET: return "request exceeds the HBM budget";
    case TL_E_NONFINITE: return "non-finite input or iterate";
  }
  return "unknown status";
}

tl_status tl_lattice_create(const tl_lattice_desc* desc, void* hip_stream, tl_lattice** out) {
  if (!desc || !out) return TL_E_INVAL;
  *out = nullptr;
  const int nx = desc->nx, ny = desc->ny;
  if (nx < 2 || ny < 2) return TL_E_INVAL;
  if ((long long)nx * ny > (1ll << 31)) return TL_E_INVAL;
  int E = desc->set_edge;
  if (E != 0 && E != 16 && E != 32 && E != 64) return TL_E_INVAL;
  const size_t nn = (size_t)nx * ny;
  if (!desc->ptrs_on_device) {
    if (desc->ea) {
      for (size_t n = 0; n < 3 * nn; ++n) {
        const float v = desc->ea[n];
        if (!(v >= 0.0f) || !std::isfinite(v)) return TL_E_INVAL;
      }
    }
    size_t nfix = 0;
    if (desc->fixed) {
      for (size_t n = 0; n < nn; ++n) nfix += desc->fixed[n] != 0;
    } else {
      nfix = (size_t)ny;
    }
    if (nfix < 2) return TL_E_INVAL;
    // every free node's own 2 x 2 block (its rods' k n n^T) must be regular
    auto rod = [&](int d, int i, int j) -> double {
      if (i < 0 || i >= nx || j < 0 || j >= ny) return 0.0;
      const bool gone = d == 0 ? i == nx - 1 : d == 1 ? j == ny - 1 : (i == 0 || j == ny - 1);
      if (gone) return 0.0;
      return desc->ea ? (double)desc->ea[(size_t)d * nn + (size_t)j * nx + i] : 1.0;
    };
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const bool fx = desc->fixed ? desc->fixed[(size_t)j * nx + i] != 0 : i == 0;
        if (fx) continue;
        const double ka = rod(0, i, j) + rod(0, i - 1, j);
        const double kb = rod(1, i, j) + rod(1, i, j - 1);
        const double kc = rod(2, i, j) + rod(2, i + 1, j - 1);
        const double dxx = ka + 0.25 * (kb + kc), dyy = 0.75 * (kb + kc);
        const double dxy = 0.43301270189221932338 * (kb - kc);
        const double tr = dxx + dyy, det = dxx * dyy - dxy * dxy;
        if (!(tr > 0.0) || !(det > 1e-12 * tr * tr)) return TL_E_INVAL;
      }
    if (desc->u_fixed)
      for (size_t n = 0; n < 2 * nn; ++n)
        if (!std::isfinite(desc->u_fixed[n])) return TL_E_NONFINITE;
  }
  // (the lookup also reads the tuning table's file on its first use, so that
  // later solves on the lattice find the table in memory)
  const int tuned_E = tuned_set_edge(nx, ny);
  if (E == 0) E = tuned_E;
  if (E == 0) E = default_set_edge(nx, ny);
  hipStream_t st = (hipStream_t)hip_stream;
  tl_lattice* L = new (std::nothrow) tl_lattice();
  if (!L) return TL_E_NOMEM;
  L->g = make_geo(nx, ny, E);
  auto fail = [&](tl_status s) { tl_lattice_destroy(L); return s; };
  if (hipGetDevice(&L->device) != hipSuccess) return fail(TL_E_DEVICE);
  const size_t np = padded_nodes(L->g);
  auto dalloc = [&](void** p, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) {
      L->allocs.push_back(*p);
      L->bytes += bytes;
      e = hipMemset(*p, 0, bytes);
    }
    return e;
  };
  void* p;
  hipError_t e;
  if ((e = dalloc(&p, 3 * np * sizeof(float))) != hipSuccess) return fail(from_hip(e));
  L->ea = (float*)p;
  if ((e = dalloc(&p, np)) != hipSuccess) return fail(from_hip(e));
  L->mask = (uint8_t*)p;
  if ((e = dalloc(&p, (size_t)L->g.M * 36 * sizeof(double))) != hipSuccess) return fail(from_hip(e));
  L->g1 = (double*)p;
  int* stats;
  if ((e = dalloc(&p, 3 * sizeof(int))) != hipSuccess) return fail(from_hip(e));
  stats = (int*)p;
  if ((e = dalloc(&p, residual_partials(L->g) * sizeof(double))) != hipSuccess) return fail(from_hip(e));
  L->res_part = (double*)p;
  if ((e = dalloc(&p, 5 * sizeof(double))) != hipSuccess) return fail(from_hip(e));
  L->res_out = (double*)p;
  if (hipHostMalloc((void**)&L->out5_host, 5 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(TL_E_NOMEM);
  // stage host inputs on the device
  const float* ea_src = desc->ea;
  const uint8_t* fx_src = desc->fixed;
  void* tmp_ea = nullptr;
  void* tmp_fx = nullptr;
  if (!desc->ptrs_on_device) {
    if (desc->ea) {
      if (hipMalloc(&tmp_ea, 3 * nn * sizeof(float)) != hipSuccess) return fail(TL_E_NOMEM);
      if (hipMemcpy(tmp_ea, desc->ea, 3 * nn * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(tmp_ea);
        return fail(TL_E_DEVICE);
      }
      ea_src = (const float*)tmp_ea;
    }
    if (desc->fixed) {
      if (hipMalloc(&tmp_fx, nn) != hipSuccess) { if (tmp_ea) (void)hipFree(tmp_ea); return fail(TL_E_NOMEM); }
      if (hipMemcpy(tmp_fx, desc->fixed, nn, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(tmp_fx);
        if (tmp_ea) (void)hipFree(tmp_ea);
        return fail(TL_E_DEVICE);
      }
      fx_src = (const uint8_t*)tmp_fx;
    }
  }
  e = launch_pad_copy_stats(L->g, ea_src, fx_src, ea_src == nullptr, fx_src == nullptr, L->ea,
                            L->mask, stats, st);
  int hs[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (tmp_ea) (void)hipFree(tmp_ea);
  if (tmp_fx) (void)hipFree(tmp_fx);
  if (e != hipSuccess) return fail(from_hip(e));
  if (hs[0] != 0 || hs[1] < 2 || hs[2] != 0) return fail(TL_E_INVAL);
  if (desc->u_fixed) {
    if ((e = dalloc(&p, nn * sizeof(double2))) != hipSuccess) return fail(from_hip(e));
    L->ufix = (double2*)p;
    e = hipMemcpy(L->ufix, desc->u_fixed, nn * sizeof(double2),
                  desc->ptrs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(from_hip(e));
  }
  // Coarse space of the upper-level preconditioner: aggregates of whole
  // upper-level workgroups (at most AGG_MAX of them), centroids on the host;
  // none when its LDS would not fit beside the upper-level windows.
  if (coarse_shape(L->g).two_level) {
    const CoarseShape cs = coarse_shape(L->g);
    const int M = L->g.M;
    const AggLayout al = agg_layout(M, L->g.mx, cs.nwg);
    L->agg_nwg = cs.nwg;
    L->agg_g = al.g;
    L->agg_sets = al.sets;
    L->naggr = al.naggr;
    std::vector<double> xy(2 * (size_t)L->naggr, 0.0);
    std::vector<int> cnt(L->naggr, 0);
    for (int sidx = 0; sidx < M; ++sidx) {
      const int I = sidx % L->g.mx, J = sidx / L->g.mx, E = L->g.E;
      const int i0 = I * E, j0 = J * E;
      const int tw = std::min(E, L->g.nx - i0), th = std::min(E, L->g.ny - j0);
      const double ic = i0 + 0.5 * (tw - 1), jc = j0 + 0.5 * (th - 1);
      const int a = sidx / L->agg_sets;
      xy[2 * a] += ic + 0.5 * jc;
      xy[2 * a + 1] += jc * 0.86602540378443864676;
      ++cnt[a];
    }
    for (int a = 0; a < L->naggr; ++a) {
      xy[2 * a] /= cnt[a];
      xy[2 * a + 1] /= cnt[a];
    }
    const size_t n = 6 * (size_t)L->naggr;
    if ((e = dalloc(&p, n * n * sizeof(double))) != hipSuccess) return fail(from_hip(e));
    L->agg_inv = (double*)p;
    if ((e = dalloc(&p, xy.size() * sizeof(double))) != hipSuccess) return fail(from_hip(e));
    L->agg_xy = (double*)p;
    if ((e = hipMemcpy(L->agg_xy, xy.data(), xy.size() * sizeof(double), hipMemcpyHostToDevice)) !=
        hipSuccess)
      return fail(from_hip(e));
  }
  e = launch_group1(L->g, L->ea, L->mask, L->g1, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(from_hip(e));
  *out = L;
  return TL_OK;
}

void tl_lattice_destroy(tl_lattice* L) {
  if (!L) return;
  for (int k = 0; k < 2; ++k)
    if (L->work[k]) {
      L->work[k]->release();
      delete L->work[k];
    }
  for (void* p : L->allocs) (void)hipFree(p);
  if (L->out5_host) (void)hipHostFree(L->out5_host);
  delete L;
}

tl_status tl_lattice_get_facts(const tl_lattice* L, tl_lattice_facts* out) {
  if (!L || !out) return TL_E_INVAL;
  out->nx = L->g.nx;
  out->ny = L->g.ny;
  out->set_edge = L->g.E;
  out->sets_x = L->g.mx;
  out->sets_y = L->g.my;
  out->sets = L->g.M;
  out->dof = 2ll * L->g.nx * L->g.ny;
  out->device_bytes = (int64_t)L->bytes;
  out->solve_bytes[0] = (int64_t)work_bytes(L->g, false, 20001);
  out->solve_bytes[1] = (int64_t)work_bytes(L->g, true, 20001);
  return TL_OK;
}

tl_status tl_solve(tl_lattice* L, const double* f_dev, double* u_dev, const tl_opts* opts,
                   tl_info* info, void* hip_stream) {
  if (!L || !f_dev || !u_dev) return TL_E_INVAL;
  Opts o;
  if (resolve_opts(opts, &o) != TL_OK) return TL_E_INVAL;
  apply_tuned(L, &o);
  std::lock_guard<std::mutex> lock(L->mu);
  tl_status err = ensure_band(L, o, (hipStream_t)hip_stream);
  if (err != TL_OK) return err;
  Work* w = lattice_work(L, o.mixed, o.max_iters + 1, &err);
  if (!w) return err;
  return run_solve(L, w, o, f_dev, u_dev, info, (hipStream_t)hip_stream, w->ctrl_host, true);
}

tl_status tl_residual(tl_lattice* L, const double* f_dev, const double* u_dev, double* r_dev,
                      double out[3], void* hip_stream) {
  if (!L || !f_dev || !u_dev || !out) return TL_E_INVAL;
  std::lock_guard<std::mutex> lock(L->mu);
  return certify(L, f_dev, u_dev, r_dev, out, (hipStream_t)hip_stream);
}

}  // extern "C"
