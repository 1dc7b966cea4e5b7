// Host-side runtime structures shared by the single-solve, batch and server
// paths.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "tl.h"
#include "tl_internal.h"

namespace tl {

// Device state of one solve (allocated once per lattice and precision, or
// per server request).
struct Work {
  Geo g{};
  bool mixed = false;
  int hist_cap = 0;
  size_t bytes = 0;
  double2* u[2] = {nullptr, nullptr};
  void* d[2] = {nullptr, nullptr};
  double *a = nullptr, *krow = nullptr, *force = nullptr, *nrm = nullptr, *off = nullptr;
  double *bdiag = nullptr, *binv = nullptr;
  double *cr = nullptr, *cu = nullptr, *cw = nullptr, *cz = nullptr, *cq = nullptr;
  double *cs = nullptr, *cp = nullptr, *cn = nullptr, *pub0 = nullptr, *pub1 = nullptr;
  double* pub2 = nullptr;
  double *red = nullptr, *hist = nullptr;
  Ctrl* ctrl = nullptr;
  unsigned* flags = nullptr;       // grid-sum arrival flags of the upper-level kernel
  Ctrl* ctrl_host = nullptr;       // pinned
  std::vector<void*> allocs;
  std::vector<hipEvent_t> events;  // kernel timing (opts.profile), 4 per iteration of a chunk

  tl_status alloc(const Geo& g, bool mixed, int hist_cap);
  void release();
};

struct Opts {
  bool mixed;
  double rtol;
  int max_iters;
  int inner;
  int overlap;           // relaxation region widened by this many nodes
  int coarse_iters;
  double coarse_rtol;
  int warm;
  tl_trace* trace;
  int profile;
  bool exact;            // exact local solves with the lattice's band factors
  bool overlap_default;  // the caller left overlap at 0 (library default or tuned)
  bool inner_default;    // the caller left inner_iters at 0
};

}  // namespace tl

struct tl_lattice {
  tl::Geo g{};
  int device = 0;
  float* ea = nullptr;          // padded [3][ny + 2][pitch]
  uint8_t* mask = nullptr;      // padded [ny + 2][pitch]
  double2* ufix = nullptr;      // [ny][nx] prescribed displacements, or null (= 0)
  double* g1 = nullptr;         // [M][36]
  size_t bytes = 0;
  std::vector<void*> allocs;
  std::mutex mu;
  tl::Work* work[2] = {nullptr, nullptr};
  double* res_part = nullptr;   // certification scratch
  double* res_out = nullptr;
  double* out5_host = nullptr;  // pinned
  // coarse space of the upper-level preconditioner (built on first solve)
  double* agg_inv = nullptr;    // [6 naggr][6 naggr]
  double* agg_xy = nullptr;     // [naggr][2] aggregate centroids
  int naggr = 0, agg_sets = 0, agg_g = 0, agg_nwg = 0;
  bool agg_ready = false;
  std::mutex agg_mu;
  // band Cholesky factors of the sets' relaxation regions, by overlap 0, 1,
  // 2, 4 (built on the first exact solve with that overlap)
  double* band[4] = {nullptr, nullptr, nullptr, nullptr};
  std::mutex band_mu;
};

namespace tl {

int default_set_edge(int nx, int ny);
Geo make_geo(int nx, int ny, int E);
size_t padded_nodes(const Geo& g);
size_t work_bytes(const Geo& g, bool mixed, int hist_cap);
struct CoarseShape {
  int nwg, vec_lds, blk_lds;
  int two_level;      // the coarse space's LDS fits beside the windows
};
CoarseShape coarse_shape(const Geo& g);
tl_status resolve_opts(const tl_opts* o, Opts* r);
int default_inner_iters(int E, bool mixed);
// Autotuning table (tl_tune.cpp): the tuned set edge of a shape (0: none),
// and the tuned overlap and sweeps of the lattice's shape and the solve's
// precision where the caller left them at 0 and the entry's set edge is the
// lattice's.
int tuned_set_edge(int nx, int ny);
// The lattice's band factors for the solve's overlap, built on first use
// (synchronises the stream when it builds them); TL_E_INVAL where exact
// local solves are not supported (float32 form, 64 x 64 sets).
tl_status ensure_band(tl_lattice* L, const Opts& o, hipStream_t st);
void apply_tuned(const tl_lattice* L, Opts* o);
// Build the lattice's upper-level coarse space once (needs one solve state
// just initialised by its init kernel); synchronises the stream.
tl_status ensure_coarse_space(tl_lattice* L, Work* w, const Opts& o, const double* f,
                              hipStream_t st);
void make_iteration_args(const tl_lattice* L, Work* w, const Opts& o, const double* f,
                         TileArgs* ta, OffArgs* oa, BlockArgs* ba, CoarseArgs* ca);
tl_status enqueue_iteration(const tl_lattice* L, Work* w, const Opts& o, const double* f,
                            hipStream_t st, hipEvent_t* ev = nullptr);
// The lattice's cached work space for one precision (caller holds L->mu).
Work* lattice_work(tl_lattice* L, bool mixed, int hist_cap, tl_status* err);
// One solve on a prepared work space.  ctrl_host receives the control block
// between chunks (pinned memory, or any host memory); with use_events = false
// no HIP event is created (no kernel timing; info->ms is host wall time).
tl_status run_solve(tl_lattice* L, Work* w, const Opts& o, const double* f, double* u,
                    tl_info* info, hipStream_t st, Ctrl* ctrl_host, bool use_events);
tl_status certify(const tl_lattice* L, const double* f, const double* u, double* r,
                  double out3[3], hipStream_t st);

// Process-wide admission of persistent upper-level grids on the current
// device.  Every workgroup of such a grid must be resident at once (its grid
// sums wait on all of them), so two grids enqueued on different streams by
// different calls must not each be left partly resident.  Workgroups are
// dispatched round-robin over the XCDs, so a grid of n workgroups places at
// most ceil(n / XCDs) on any one; counting each as a whole CU, grids run
// together only while those counts fit an XCD's CUs, and a grid that needs
// more (a fused batch at two workgroups per CU) runs alone.  The guard is
// held from the enqueue of a chunk of iterations until the host has seen
// that chunk finish: its destructor synchronises `stream` before releasing.
class PersistentGuard {
 public:
  PersistentGuard(int nwg, hipStream_t stream);
  ~PersistentGuard();
  PersistentGuard(const PersistentGuard&) = delete;
  PersistentGuard& operator=(const PersistentGuard&) = delete;

 private:
  int dev_ = -1;
  int demand_ = 0;
  hipStream_t stream_ = nullptr;
};

}  // namespace tl
