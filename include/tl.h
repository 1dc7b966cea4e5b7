/*
 * tl.h -- C ABI of the MI355X hierarchical lattice solver.
 *
 * The library solves the linear equations K u = f of a 2-D triangle-lattice
 * truss (Xu, Liu, Dong, "Scalable hierarchical parallel algorithm for the
 * solution of super large-scale sparse linear equations"; problem statement
 * Eq. 1, test problem section 3.1) with the paper's hierarchical iteration:
 * per-set local relaxation with the neighbouring sets' displacements held
 * fixed (section 2.2, Eq. 11-14), an upper-level ("master") equilibrium
 * correction over q = 9 incremental modes per set (Eq. 3-10), and the global
 * relative-residual stop test (Eq. 19).  Sets are E x E node tiles of the
 * lattice's index grid, one GPU workgroup each.
 *
 * Lattice and layouts
 *   Node (i, j), 0 <= i < nx, 0 <= j < ny, sits at (i + j/2, j*sqrt(3)/2).
 *   Every node stores its three forward rods, length 1:
 *     d = 0 : (i, j)-(i+1, j)   d = 1 : (i, j)-(i, j+1)   d = 2 : (i, j)-(i-1, j+1)
 *   ea      : float  [3][ny][nx], axial stiffness EA of each rod (element
 *             stiffness (EA/L) n n^T, L = 1); entries of rods that would
 *             leave the lattice are ignored.
 *   fixed   : uint8  [ny][nx], nonzero = node clamped (both DOFs prescribed).
 *   u_fixed : double [ny][nx][2], prescribed displacement of clamped nodes.
 *   f, u    : double [ny][nx][2], loads and displacements, C order, x then y.
 *             Loads on clamped DOFs are ignored (they are support reactions).
 *
 * Ownership and threading
 *   All pointers in a call are borrowed for the duration of the call only,
 *   except that tl_submit borrows f_dev and u_dev until tl_poll has reported
 *   the request finished.  Host arrays passed to tl_lattice_create are copied.
 *   A lattice is immutable after creation; solves on one lattice from several
 *   host threads are serialised internally.  Device pointers are hipMalloc'd
 *   (or PyTorch) memory on the current device.
 *
 * Concurrency across streams
 *   The upper-level kernel is a persistent grid whose workgroups must all be
 *   resident at once.  Calls from several host threads (tl_solve on different
 *   lattices or streams, tl_solve_batch, the server's worker) are admitted
 *   process-wide: their persistent grids run together only while all of
 *   their workgroups fit the device's CUs together, else one after another,
 *   one chunk of outer iterations at a time.  Results do not depend on this.
 *
 * Errors
 *   Every call returns a tl_status; nothing aborts or throws across the ABI.
 *   TL_E_NOCONV still writes the last iterate to u and fills the tl_info.
 *
 * Environment (tuning and diagnostics; read at each call, unset = default)
 *   TL_TUNE_CACHE          file of measured set edges, overlaps and sweeps
 *                          (tl_tune, below).
 *   TL_TILE_THREADS        threads of the tile kernel where the set edge
 *                          allows several: 256/512/1024 for 32 x 32 sets
 *                          without overlap, 256/512 with it, 512/1024 for
 *                          64 x 64; other values keep the default.
 *   TL_COARSE_SETS_PER_WG  sets per upper-level workgroup (default 16).
 *   TL_COARSE_2LEVEL       0: no aggregate coarse space in the upper-level
 *                          preconditioner (block Jacobi alone).
 *   TL_COARSE_NO_LDS       1: upper-level vectors and blocks stay in HBM.
 *   TL_COARSE_WARM         0: the upper-level PCG starts from zero instead
 *                          of the previous coefficients.
 *   TL_COARSE_REF          1: its tolerance is relative to the zero-start
 *                          residual instead of the initial one.
 *   TL_COARSE_BATCH_WG     cap on co-resident workgroups of the fused
 *                          upper-level kernel (for profilers that keep part
 *                          of the device); results do not change.
 *   None of these changes the method; each changes only how the work is
 *   laid out or how far the upper-level PCG iterates.
 */
#ifndef TL_H
#define TL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tl_lattice tl_lattice;   /* opaque */
typedef struct tl_server tl_server;     /* opaque */

typedef enum {
    TL_OK = 0,
    TL_PENDING = 1,        /* tl_poll: request not finished yet               */
    TL_E_INVAL = -1,       /* bad argument or descriptor                        */
    TL_E_NOMEM = -2,       /* device allocation failed                          */
    TL_E_NOCONV = -3,      /* max_iters reached before the tolerance            */
    TL_E_DEVICE = -4,      /* HIP runtime error or a device-side abort          */
    TL_E_BUDGET = -5,      /* request can never fit the server's HBM budget, or a
                              lattice's upper-level workgroups cannot all be
                              co-resident on the device                         */
    TL_E_NONFINITE = -6    /* non-finite input or iterate                        */
} tl_status;

typedef enum {
    TL_FP64 = 0,           /* every stage in float64                            */
    TL_MIXED = 1           /* relaxation sweeps in float32 with per-set 2^-e
                              scaling; residual, upper level, update in float64 */
} tl_precision;

typedef enum {
    TL_LOCAL_PCG = 0,      /* relaxation by preconditioned-CG sweeps (default)    */
    TL_LOCAL_EXACT = 1     /* exact relaxation with the regions' band Cholesky
                              factors, built once per lattice and overlap     */
} tl_local_solve;

typedef struct {
    int32_t nx, ny;            /* nodes per side, each >= 2                      */
    const float* ea;           /* [3][ny][nx]; NULL = every rod EA 1             */
    const uint8_t* fixed;      /* [ny][nx]; NULL = nodes with i == 0 clamped      */
    const double* u_fixed;     /* [ny][nx][2]; NULL = 0                          */
    int32_t set_edge;          /* E in {16, 32, 64}; 0 = chosen by the library    */
    int32_t ptrs_on_device;    /* 1: ea/fixed/u_fixed are device pointers         */
} tl_lattice_desc;

/* Optional per-solve diagnostics: device buffers (any may be NULL) that
 * receive the quantities of the last completed outer iteration whose
 * upper-level system was solved.  Sizes use M = number of sets. */
typedef struct {
    double* delta;        /* [ny][nx][2] relaxation increment (mode 7, Eq. 13), as stored */
    double* kdiag;        /* [M][9][9]  diagonal upper-level blocks (Eq. 6)            */
    double* koff;         /* [M][6][9][9] blocks to the 6 neighbouring sets (Eq. 6),
                             neighbour order (+1,0) (0,+1) (-1,+1) (-1,0) (0,-1) (+1,-1) */
    double* force;        /* [M][9] upper-level force (Eq. 7)                          */
    double* coef;         /* [M][9] coefficients a (Eq. 8)                             */
    double* residual_history; /* [max_iters + 1]: max(R1, R2) per outer iteration      */
} tl_trace;

typedef struct {
    tl_precision precision;
    double rtol;               /* stop when max(R1, R2) <= rtol (Eq. 19, both norms) */
    int32_t max_iters;         /* outer iterations; 0 = library default             */
    int32_t inner_iters;       /* relaxation PCG sweeps per set; 0 = default: 24
                                  with 64 x 64 sets, 20 for float64 with 32 x 32
                                  sets, else 16                                     */
    int32_t coarse_iters;      /* upper-level PCG iteration cap; 0 = default: 100;
                                  200 for lattices of 16384 sets or more; 20
                                  (TL_FP64) or 25 (TL_MIXED) for lattices of at
                                  most 256 sets                                     */
    double coarse_rtol;        /* upper-level PCG relative tolerance; 0 = default:
                                  0.05 for lattices of 16384 sets or more, else 0.15
                                  for float64 with sets of at most 32 x 32, else 0.1 */
    int32_t warm_start;        /* 1: start from the free DOFs of u (else from 0)     */
    tl_trace* trace;           /* NULL, or diagnostics to fill                       */
    int32_t profile;           /* 1: time every kernel launch with HIP events on the
                                  solve's stream (fills the *_ms fields of tl_info);
                                  N > 1: only the launches of every N-th iteration  */
    int32_t overlap;           /* relax each set on its tile widened by this many
                                  nodes on every side, keeping the increment on the
                                  set (section 2.2 end): 1, 2 or 4; -1 = the set
                                  alone; 0 = library default (2)                    */
    int32_t local_solve;       /* a tl_local_solve.  TL_LOCAL_PCG (0): relaxation by
                                  inner_iters PCG sweeps (default).  TL_LOCAL_EXACT
                                  (1): exact (section 2.2 end): each set's region
                                  stiffness k^Inner is factored once (band Cholesky)
                                  on the first such solve of the lattice and
                                  overlap, kept with the lattice and reused; that
                                  first call, batched or served too, synchronises
                                  its stream once.  Float64 form only, sets of at
                                  most 32 x 32 nodes; else TL_E_INVAL.  The factors
                                  take about 64 (E + 2w)^3 bytes per set, counted
                                  in tl_lattice_facts.device_bytes; TL_E_NOMEM when
                                  they do not fit                                  */
} tl_opts;

typedef struct {
    tl_status status;
    int32_t iters;             /* outer iterations performed                      */
    double rel_res_l1;         /* Eq. 19 1-norm relative residual of the returned u */
    double rel_res_l2;         /* 2-norm relative residual of the returned u        */
    double energy;             /* total energy Pi of Eq. 2 at the returned u        */
    double ms;                 /* device time of the solve                         */
    int64_t coarse_iters;      /* upper-level PCG iterations summed over the solve  */
    double tile_ms;            /* with opts->profile: summed duration of the tile
                                  (update/residual/relaxation) kernel launches     */
    double offdiag_ms;         /* ... of the boundary-block kernel launches         */
    double coarse_ms;          /* ... of the upper-level kernel launches            */
    int32_t tile_launches;     /* launches those sums cover (iterations that ran,
                                  every N-th with profile = N).  tl_solve_batch
                                  with opts->profile: tile_ms and tile_launches
                                  cover the fused tile launches of the lattice's
                                  set edge while at least one lattice of that
                                  edge was still iterating; offdiag_ms and
                                  coarse_ms cover the whole call                   */
} tl_info;

/* Lattice geometry facts (for sizing buffers). */
typedef struct {
    int32_t nx, ny, set_edge, sets_x, sets_y, sets;
    int64_t dof;               /* 2 * nx * ny                                      */
    int64_t device_bytes;      /* device memory held by the lattice                */
    int64_t solve_bytes[2];    /* per-solve state for TL_FP64, TL_MIXED            */
} tl_lattice_facts;

/* Validate the descriptor, copy the lattice to the device and precompute the
 * constant part of the upper-level diagonal blocks (translation and
 * gradient modes, Eq. 6 with Eq. 9-10).  Returns TL_E_INVAL without touching
 * the device when nx or ny < 2, fewer than two nodes are clamped, set_edge is
 * not 0/16/32/64, or an EA is negative or not finite (host-side input only);
 * and TL_E_INVAL after the copy when the same holds for device input, or when
 * a free node's own 2 x 2 stiffness block is singular (no rod, or only
 * collinear rods, hold it), since K is then not positive definite (Eq. 1
 * assumes it is).  Larger mechanisms are not detected here; a solve of such a
 * lattice ends with TL_E_NONFINITE or TL_E_NOCONV. */
tl_status tl_lattice_create(const tl_lattice_desc* desc, void* hip_stream, tl_lattice** out);
void tl_lattice_destroy(tl_lattice* lat);
tl_status tl_lattice_get_facts(const tl_lattice* lat, tl_lattice_facts* out);

/* Solve K u = f for one load vector, stream-ordered on hip_stream (NULL =
 * the null stream), returning after completion.  f_dev, u_dev: device
 * double [ny][nx][2].  Returns TL_E_NONFINITE if f has a non-finite free
 * entry or an iterate becomes non-finite. */
tl_status tl_solve(tl_lattice* lat, const double* f_dev, double* u_dev,
                   const tl_opts* opts, tl_info* info, void* hip_stream);

/* Solve n independent lattices in fused launches: per outer iteration one
 * tile launch per set edge over the sets of all lattices, one boundary-block
 * and one block-inverse launch over all sets, and one persistent upper-level
 * launch in which every lattice owns its own range of workgroups; chunks of
 * iterations are captured once in a hipGraph and replayed.  The upper-level
 * launch may hold more workgroups than fit the device at once (they take their
 * places in start order, so a lattice whose workgroups have all started runs
 * to its end); each lattice's own upper-level workgroups must fit at once
 * (else TL_E_BUDGET).  Each lattice's result is bit for
 * bit the one tl_solve gives it alone (its kernels, set edge and reduction
 * orders depend on that lattice only).  infos[k] receives lattice k's result
 * (ms = wall time from the call's start until lattice k's finish was seen at
 * the end of a chunk of iterations: its latency within the batch); the return
 * value is TL_OK when every lattice converged, else the first failing status.
 * With opts->profile the chunks are not captured: every launch is timed with
 * HIP events (see tl_info) and the control blocks are read after every outer
 * iteration, so such a call is slower than an unprofiled one. */
tl_status tl_solve_batch(int32_t n, tl_lattice* const* lats, const double* const* f_dev,
                         double* const* u_dev, const tl_opts* opts, tl_info* infos,
                         void* hip_stream);

/* r = f - K u (float64; the bracket of Eq. 7) into r_dev (may be NULL), and
 * out[0..2] = R1, R2 (Eq. 19, relative to the constrained right-hand side
 * f - K_fc u_c) and the energy Pi (Eq. 2) of u. */
tl_status tl_residual(tl_lattice* lat, const double* f_dev, const double* u_dev,
                      double* r_dev, double out[3], void* hip_stream);

/* Continuous-batching server.  Requests are admitted in arrival order while
 * the device state of all admitted requests fits hbm_budget_bytes, fewer than
 * max_slots are admitted; a background worker advances all
 * admitted requests of a precision together in fused launches, eight outer
 * iterations at a time, retires each as it converges and admits waiting
 * requests at once.  Results are bit for bit those of tl_solve alone.
 * tl_submit returns TL_E_BUDGET for a request that could never be admitted.
 * It records an event on hip_stream (NULL = the null stream): the request's
 * kernels wait for the work enqueued there before the call, so f_dev may be
 * produced by a kernel that has not finished yet.  u_dev is complete when
 * tl_poll reports the request finished. */
tl_status tl_server_create(size_t hbm_budget_bytes, int32_t max_slots, tl_server** out);
tl_status tl_submit(tl_server* srv, tl_lattice* lat, const double* f_dev, double* u_dev,
                    const tl_opts* opts, void* hip_stream, uint64_t* ticket);
/* TL_PENDING until the request has finished; then its final status, with
 * out filled (out->ms = submit-to-finish wall time). */
tl_status tl_poll(tl_server* srv, uint64_t ticket, tl_info* out);
/* Waits for every admitted and queued request, then frees the server. */
void tl_server_destroy(tl_server* srv);

const char* tl_strerror(tl_status s);

/* Autotuning of the launch choices of a lattice shape: the set edge E of the
 * partition into sets (section 2.2), the overlap of the relaxation region
 * (section 2.2 end) and the relaxation sweeps per set (the inner solve of
 * Eq. 12).  A process-wide table maps a shape key and a precision to one
 * choice.  The key is (round(2 log2 nx), round(2 log2 ny)): lattices whose
 * sides fall in the same half-octaves share an entry.  The table is read from
 * the text file named by the environment variable TL_TUNE_CACHE at its first
 * use (a missing file is an empty table), and tl_tune rewrites that file after
 * every measurement.
 *
 * How the library applies it: tl_lattice_create with set_edge = 0 takes the
 * set edge of the shape's mixed-precision entry, else of its float64 entry,
 * else the built-in rule.  A solve (tl_solve, tl_solve_batch, tl_submit,
 * tl_solve_noalloc) whose opts leave overlap or inner_iters at 0 takes them
 * from the entry of the lattice's shape and the solve's precision when that
 * entry's set edge is the lattice's, else the built-in defaults.  The choice
 * depends on the lattice's shape and the precision alone, so a lattice's
 * batched and served results stay bit for bit those of tl_solve alone, as
 * long as the table does not change between the calls. */
typedef struct {
    int32_t set_edge;          /* 16, 32 or 64; 0 = no entry                      */
    int32_t overlap;           /* -1 (the set alone), 1, 2 or 4                    */
    int32_t inner_iters;       /* relaxation sweeps per set                        */
    int32_t nx, ny;            /* the lattice the choice was measured on           */
    double ms;                 /* its measured solve time                          */
} tl_tune_entry;

/* Measure candidate choices on the lattice of desc (arrays as for
 * tl_lattice_create) with the load f_dev (device double [ny][nx][2]) in
 * opts->precision to opts->rtol (other opts fields as for tl_solve; overlap,
 * inner_iters and desc->set_edge are the searched quantities and ignored),
 * and record the fastest choice that converged under the shape's key.  The
 * search is coordinate-wise from the built-in defaults: the set edge over
 * {16, 32, 64} (edges at most the lattice's longer side), then the overlap
 * over {1, 2, 4}, then the sweeps over the default +-4 and +-8; each
 * candidate is solved twice after a warm-up and timed by host wall clock
 * (the faster of the two counts).  Allocates device memory for the candidate
 * lattices and one displacement array; runs on hip_stream.  out receives the
 * choice.  Returns TL_E_NOCONV when no candidate converged (nothing recorded). */
tl_status tl_tune(const tl_lattice_desc* desc, const double* f_dev, const tl_opts* opts,
                  tl_tune_entry* out, void* hip_stream);
/* The table's entry for a shape and precision (out->set_edge = 0: none). */
tl_status tl_tune_lookup(int32_t nx, int32_t ny, tl_precision precision, tl_tune_entry* out);
/* Merge the entries of a table file into the table (TL_E_INVAL on a malformed
 * file, nothing merged), write the table to a file, or empty it. */
tl_status tl_tune_load(const char* path);
tl_status tl_tune_save(const char* path);
tl_status tl_tune_clear(void);

/* tl_solve without any device or host allocation, for callers that cannot
 * allocate (code that must not call hipMalloc, tight serving loops, harnesses
 * that forbid allocation).  The solve state lives in a fixed, library-owned
 * device array of TL_NOALLOC_SCRATCH_BYTES per GPU (held until the process
 * ends), which every tl_solve_noalloc call on that GPU reuses: calls on one
 * GPU are serialised internally, and the array keeps the last call's
 * contents (everything a solve reads is cleared by the solve itself).
 * Results are bit for bit those of tl_solve.  Returns TL_E_BUDGET, before
 * touching the device, when the lattice's solve state for opts (the
 * solve_bytes of tl_lattice_facts, with max_iters + 1 history entries) exceeds
 * the array; TL_E_INVAL for opts->profile or opts->trace (both would need
 * allocations).  info->ms is host wall time.  The lattice itself was
 * allocated by tl_lattice_create. */
#define TL_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
tl_status tl_solve_noalloc(tl_lattice* lat, const double* f_dev, double* u_dev,
                           const tl_opts* opts, tl_info* info, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* TL_H */
