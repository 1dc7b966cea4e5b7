// tl_solve_noalloc: tl_solve with its solve state in a fixed device array.
//
// For callers that cannot allocate: the work space that tl_solve allocates
// once per lattice and precision (displacement and increment ping-pong
// buffers, the upper-level blocks and PCG vectors, grid-sum slots, control
// block) is carved instead from `scratch`, a file-scope device array of
// TL_NOALLOC_SCRATCH_BYTES that each GPU holds until the process ends.  The
// array's host-side name is not a device address: its address on each device
// is taken once, with that device current, by hipGetSymbolAddress and kept
// per device; only that pointer is ever passed to kernels.
//
// Every call on a device reuses the same array and leaves its contents
// behind, so each call clears what its kernels read before writing: the
// padded displacement and increment buffers in full (the stencil reads their
// padding ring), then the initial state, coefficients, barrier counters and
// control block as tl_solve does.  Calls on one device are serialised by a
// host mutex; nothing here allocates memory, creates events or streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "tl.h"
#include "tl_internal.h"
#include "tl_runtime.h"

// The solve state of every tl_solve_noalloc call on a device.
static __device__ __align__(256) unsigned char scratch[TL_NOALLOC_SCRATCH_BYTES];

namespace tl {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_dev_mu[kMaxDevices];         // serialises the calls on one device
void* g_scratch_ptr[kMaxDevices] = {};    // device address of `scratch`, per device

// Zero n 16-byte words (a fill kernel rather than a memset, so the clear is
// an ordinary kernel in the stream).
__global__ __launch_bounds__(256) void k_zero16(double2* p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += stride)
    p[e] = make_double2(0.0, 0.0);
}

constexpr size_t kAlign = 256;
size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Point w's buffers into [base, base + carve_bytes).  The displacement and
// increment buffers come first, contiguous, so one fill clears them.
void carve(Work* w, unsigned char* base, const Geo& g, bool mixed, int hist_cap,
           size_t* node_bytes) {
  const size_t np = padded_nodes(g), M = g.M;
  unsigned char* p = base;
  auto take = [&](size_t bytes) {
    unsigned char* q = p;
    p += align_up(bytes);
    return (void*)q;
  };
  w->g = g;
  w->mixed = mixed;
  w->hist_cap = hist_cap;
  for (int k = 0; k < 2; ++k) w->u[k] = (double2*)take(np * sizeof(double2));
  for (int k = 0; k < 2; ++k) w->d[k] = take(np * (mixed ? sizeof(float2) : sizeof(double2)));
  *node_bytes = (size_t)(p - base);
  w->a = (double*)take(M * Q * sizeof(double));
  w->krow = (double*)take(M * KROW * sizeof(double));
  w->force = (double*)take(M * Q * sizeof(double));
  w->nrm = (double*)take(M * NRM * sizeof(double));
  w->off = (double*)take(M * NDIR * Q * Q * sizeof(double));
  w->bdiag = (double*)take(M * Q * Q * sizeof(double));
  w->binv = (double*)take(M * Q * Q * sizeof(double));
  double** vecs[] = {&w->cr, &w->cu, &w->cw, &w->cz, &w->cq, &w->cs, &w->cp, &w->cn,
                     &w->pub0, &w->pub1, &w->pub2};
  for (double** v : vecs) *v = (double*)take(M * Q * sizeof(double));
  w->red = (double*)take(2 * COARSE_MAX_WG * REDW * sizeof(double));
  w->hist = (double*)take((size_t)hist_cap * sizeof(double));
  w->ctrl = (Ctrl*)take(sizeof(Ctrl));
  w->flags = (unsigned*)take(COARSE_MAX_WG * sizeof(unsigned));
  w->bytes = (size_t)(p - base);
}

// Bytes of the carved work space (the layout above, from address 0).
size_t carve_bytes(const Geo& g, bool mixed, int hist_cap) {
  Work w;
  size_t node_bytes = 0;
  carve(&w, nullptr, g, mixed, hist_cap, &node_bytes);
  return w.bytes;
}

}  // namespace

}  // namespace tl

using namespace tl;

extern "C" tl_status tl_solve_noalloc(tl_lattice* L, const double* f_dev, double* u_dev,
                                      const tl_opts* opts, tl_info* info, void* hip_stream) {
  if (!L || !f_dev || !u_dev) return TL_E_INVAL;
  Opts o;
  if (resolve_opts(opts, &o) != TL_OK) return TL_E_INVAL;
  if (o.profile || o.trace || o.exact) return TL_E_INVAL;   // each would need allocations
  // tuned choices, as tl_solve takes them (the table was read from its file
  // when the lattice was created: this lookup allocates nothing)
  apply_tuned(L, &o);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TL_E_DEVICE;
  if (dev != L->device || dev < 0 || dev >= kMaxDevices) return TL_E_INVAL;
  const int hist_cap = o.max_iters + 1;
  if (carve_bytes(L->g, o.mixed, hist_cap) > TL_NOALLOC_SCRATCH_BYTES) return TL_E_BUDGET;
  std::lock_guard<std::mutex> dev_lock(g_dev_mu[dev]);
  if (!g_scratch_ptr[dev]) {
    // set-up, once per device with that device current: the array's device
    // address (the host-side symbol is only a stand-in for it)
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TL_E_DEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  std::lock_guard<std::mutex> lat_lock(L->mu);
  hipStream_t st = (hipStream_t)hip_stream;
  Work w;                                   // pointers only: nothing is allocated
  size_t node_bytes = 0;
  carve(&w, (unsigned char*)g_scratch_ptr[dev], L->g, o.mixed, hist_cap, &node_bytes);
  const size_t n16 = node_bytes / sizeof(double2);
  hipLaunchKernelGGL(k_zero16, dim3((unsigned)std::min<size_t>((n16 + 255) / 256, 8192)), dim3(256),
                     0, st, w.u[0], n16);
  if (hipGetLastError() != hipSuccess) return TL_E_DEVICE;
  Ctrl ctrl_host{};
  return run_solve(L, &w, o, f_dev, u_dev, info, st, &ctrl_host, false);
}
