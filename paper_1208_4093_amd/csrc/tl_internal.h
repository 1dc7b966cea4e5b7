// Internal declarations shared by the HIP kernels and the host runtime.
//
// Device layout of one lattice (nx x ny nodes, set edge E):
//   * node arrays are padded with a one-node ring: node (i, j), -1 <= i <= nx,
//     -1 <= j <= ny, lives at (j + 1) * pitch + (i + LPAD).  The ring is clamped
//     (mask 1), carries zero rod stiffness and zero displacement, so stencil
//     and halo loads never leave the allocation and need no bounds tests;
//   * ea      : float  [3][ny + 2][pitch]   rod EA of the three forward rods;
//   * mask    : uint8  [ny + 2][pitch]      1 = clamped (or ring);
//   * u, delta: double2 / T2 [ny + 2][pitch], two of each (ping-pong);
//   * per-set upper-level data, set id s = J * mx + I:
//       g1 [M][36]   constant 6x6 block of the translation/gradient modes;
//       krow [M][27] rows of modes 7-9 of the diagonal block (cols 1-9);
//       force [M][9], norm partials [M][4];
//       off [M][6][81] blocks to the six neighbouring sets;
//       bdiag [M][81], lfac [M][45], bscale [M][9]  assembled block and its
//       scaled, pivot-dropping Cholesky factor (block-Jacobi preconditioner).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tl {

constexpr int Q = 9;            // modes per set (Eq. 9, 10, 13, 14)
constexpr int NDIR = 6;         // neighbouring sets in the set grid
constexpr int KROW = 27;        // 3 relaxation-mode rows x 9 columns
constexpr int NRM = 4;          // sum|r|, sum r^2, sum|f|, sum f^2 (free DOFs)
constexpr int TILE_OUT = KROW + Q + NRM;
constexpr int COARSE_NT = 256;  // threads per upper-level workgroup
constexpr int COARSE_MAX_WG = 256;
constexpr int BAR_GROUPS = 8;     // group counters of the grid barrier (one 64-byte line each)
static_assert(BAR_GROUPS * 16 + 1 <= COARSE_MAX_WG, "barrier counters live in the flag array");
constexpr int REDW = 24;        // values per workgroup and slot of a grid sum
constexpr int AGG_MAX = 32;     // aggregates of the upper-level coarse space (at most)
constexpr int AGG_GMAX = 8;     // workgroups per aggregate (at most: COARSE_MAX_WG / AGG_MAX)
constexpr int AGG_PART = (COARSE_NT / 64) * 2 * 64;   // partial sums of the window solve (doubles)
// Dynamic LDS of one upper-level workgroup, at most: the 160 KB of a CU less
// the kernel's static arrays (grid-sum and coarse-space scratch, 7 KB).
constexpr size_t COARSE_DYN_LDS_MAX = 152 * 1024;
constexpr int LPAD = 32;        // left padding (elements) of node arrays: interior
                                // rows start on a 128-byte boundary for every type

// Set-grid neighbour offsets (dI, dJ); direction d and d + 3 are opposite.
// Aggregates of the upper-level coarse space for a lattice of M sets (mx per
// row) whose upper level runs on nwg workgroups: runs of `g` whole workgroups
// (`sets` sets), `naggr` of them, and at most `nwa_max` of them meet one
// workgroup's window of neighbour sets.
struct AggLayout {
  int g, sets, naggr, nwa_max;
};
__host__ __device__ inline AggLayout agg_layout(int M, int mx, int nwg) {
  AggLayout a;
  const int spw = (M + nwg - 1) / nwg;
  a.g = (nwg + AGG_MAX - 1) / AGG_MAX;
  a.sets = spw * a.g;
  a.naggr = (M + a.sets - 1) / a.sets;
  const int win = M < spw + 2 * mx + 2 ? M : spw + 2 * mx + 2;
  const int span = win / a.sets + 2;
  a.nwa_max = a.naggr < span ? a.naggr : span;
  return a;
}

__host__ __device__ constexpr int nb_di(int d) { return d == 0 ? 1 : d == 2 ? -1 : d == 3 ? -1 : d == 5 ? 1 : 0; }
__host__ __device__ constexpr int nb_dj(int d) { return d == 1 ? 1 : d == 2 ? 1 : d == 4 ? -1 : d == 5 ? -1 : 0; }

struct Geo {
  int nx, ny, pitch, E, mx, my, M;
};

// Device-side control block of one solve.
struct Ctrl {
  int k;             // current outer iteration (advanced by the upper-level kernel)
  int done;          // 0 running, 1 finished
  int status;        // tl_status of the finished solve
  int iters;         // outer iteration at which the solve finished
  int err;           // device-side abort (barrier time-out)
  long long coarse_iters;
  double r1, r2;     // relative residuals of the last checked iterate
  unsigned bar_count;            // unused
  unsigned bar_gen;              // generation of the last grid sum
};

template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };

struct TileArgs {
  double2* u0;           // padded displacements, ping (iteration k reads u[k & 1])
  double2* u1;           // pong
  void* d0;              // T2 padded relaxation increments, ping
  void* d1;              // pong
  const double* a;       // [M][9] coefficients of the previous upper-level solve
  const double2* f;      // [ny][nx] loads (unpadded, caller's buffer)
  double* krow;          // [M][27]
  double* force;         // [M][9]
  double* nrm;           // [M][4]
  const Ctrl* ctrl;
  int inner_iters;
  int rhs_mode;          // 1: prescribed displacements present, norms use f - K_fc u_c
  // exact local solve (float64 form): every set's band Cholesky factor of its
  // region's k^Inner, by columns and by rows, BAND_CH-column chunks staged
  // through dynamic LDS; null: preconditioned-CG sweeps
  const double* band;
  size_t band_stride;    // doubles per set (both copies)
  int band_bs;           // doubles per factor column (diagonal + lower band)
};

// Exact local solves: columns per LDS chunk of the band factor, and the
// factor's shape for a relaxation region of at most R x R nodes (R = E + 2w):
// n = 2 R^2 DOFs, lower bandwidth 2R + 1, so 2R + 2 doubles a column.  A set
// keeps the factor twice: column j of L (the forward solve's order), then row
// j of L in descending j (the backward solve's order), each BS doubles.
constexpr int BAND_CH = 64;
__host__ __device__ constexpr int band_bs(int R) { return 2 * R + 2; }
__host__ __device__ constexpr size_t band_copy_doubles(int R) { return (size_t)2 * R * R * band_bs(R); }
__host__ __device__ constexpr size_t band_set_doubles(int R) { return 2 * band_copy_doubles(R); }
// Two chunk buffers, padded by 128 doubles: a column step reads 128 entries
// past its column's start from its last lane.
__host__ __device__ constexpr size_t band_chunk_bytes(int R) {
  return ((size_t)2 * BAND_CH * band_bs(R) + 128) * sizeof(double);
}

struct CoarseArgs {
  const double* g1;      // [M][36]
  const double* krow;    // [M][27]
  const double* force;   // [M][9]
  const double* nrm;     // [M][4]
  const double* off;     // [M][6][81]
  double* bdiag;         // [M][81] assembled diagonal blocks
  double* binv;          // [M][81] their pseudo-inverses (block-Jacobi preconditioner)
  double* a;             // [9M] solution (coefficients); also the warm start
  double* cr;            // [9M] pipelined-PCG vectors, own rows only
  double* cu;
  double* cw;
  double* cz;
  double* cq;
  double* cs;
  double* cp;
  double* cn;
  // Published vectors read by neighbouring sets: the start publishes B^+ P in
  // pub0 and B^+ y in pub1; PCG iteration it publishes m in pub2 (it even)
  // or pub0 (it odd), so no workgroup overwrites a vector that a slower one
  // may still be reading (the start's pair stays untouched until every
  // workgroup has passed the first iteration's grid sum).
  double* pub0;          // [9M]
  double* pub1;          // [9M]
  double* pub2;          // [9M]
  double* red;           // [2][REDW][COARSE_MAX_WG] reduction slots (value-major)
  unsigned* flags;       // [COARSE_MAX_WG] grid-barrier counters: group g at [16 g], root at [16 BAR_GROUPS]
  double* hist;          // [max_iters + 1] max(R1, R2) per outer iteration (may be null)
  double* tr_kdiag;      // optional copies of the solved system (diagnostics)
  double* tr_koff;
  double* tr_force;
  double* tr_coef;
  Ctrl* ctrl;
  int max_iters;
  int coarse_iters;
  double coarse_rtol;
  double rtol;
  int nwg;
  int warm;              // warm-start the upper-level PCG from the previous coefficients
  int coarse_ref;        // PCG tolerance relative to 1: the zero-start residual, 0: the initial one
  // Coarse space of the PCG preconditioner (naggr = 0: block-Jacobi alone):
  // aggregates of agg_sets consecutive sets (agg_g workgroups each), six
  // affine fields per aggregate, agg_inv the pseudo-inverse of their
  // upper-level matrix ([6 naggr][6 naggr]), agg_xy their centroids.
  const double* agg_inv;
  const double* agg_xy;
  int naggr;
  int agg_sets;
  int agg_g;
  int vec_lds;           // 1: own PCG vectors in LDS
  int blk_lds;           // 1: own blocks staged in LDS
  unsigned spin_limit;
};

struct OffArgs {
  const void* d0;        // T2 padded relaxation increments (iteration k writes d[(k+1) & 1])
  const void* d1;
  double* off;           // [M][6][81]
  const Ctrl* ctrl;
};

struct BlockArgs {
  const double* g1;      // [M][36]
  const double* krow;    // [M][27]
  double* bdiag;         // [M][81] assembled diagonal blocks
  double* binv;          // [M][81] their pseudo-inverses
  const Ctrl* ctrl;
};

// One lattice of a fused (batched) launch: its geometry, arguments of every
// kernel, and its offsets in the launch-wide tile, set and workgroup ranges.
struct BatchEntry {
  Geo g;
  const float* ea;
  const uint8_t* mask;
  TileArgs ta;
  OffArgs oa;
  BlockArgs ba;
  CoarseArgs ca;
  int tile0;             // first tile in its set-edge group's tile launch
  int set0;              // first set in the launch-wide set range
  int wg0, nwg;          // upper-level workgroups
};

// Launchers (tl_kernels.hip).  All are asynchronous on `stream`.
hipError_t launch_tile(bool mixed, int ov, const Geo& g, const float* ea, const uint8_t* mask,
                       const TileArgs& a, hipStream_t stream);
bool tile_overlap_supported(int ov);
hipError_t launch_offdiag(bool mixed, const Geo& g, const float* ea, const uint8_t* mask,
                          const OffArgs& a, hipStream_t stream);
hipError_t launch_blockinv(const Geo& g, const BlockArgs& a, hipStream_t stream);
hipError_t launch_coarse(const Geo& g, const CoarseArgs& a, hipStream_t stream);
size_t coarse_lds_bytes(const Geo& g, int nwg, int vec_lds, int blk_lds, int two_level);
// Coarse space of the upper-level preconditioner: A0 = P0^T K_a P0 from the
// constant blocks (g1 and the mode 1-6 corners of off), then its
// pseudo-inverse in place.
hipError_t launch_agg_setup(const Geo& g, const double* g1, const double* off,
                            const double* agg_xy, int agg_sets, int naggr, double* A0,
                            hipStream_t stream);
// Fused launches over a batch (entries and lookup tables in device memory).
hipError_t launch_tile_batch(bool mixed, int E, int ov, const BatchEntry* B, const int* tile_lat,
                             int ntiles, bool any_band, hipStream_t stream);
hipError_t launch_offdiag_batch(bool mixed, const BatchEntry* B, const int* set_lat, int nsets,
                                hipStream_t stream);
hipError_t launch_blockinv_batch(const BatchEntry* B, const int* set_lat, int nsets,
                                 hipStream_t stream);
// ticket: a device counter at 0 (the launch leaves it at 0); max_lattice_nwg:
// the most workgroups any one lattice of the launch owns (at most the
// co-resident capacity at lds, else hipErrorInvalidValue)
hipError_t launch_coarse_batch(const BatchEntry* B, const int* wg_lat, unsigned* ticket, int nwg,
                               int max_lattice_nwg, size_t lds, hipStream_t stream);
int coarse_batch_capacity(size_t lds);   // co-resident workgroups of the fused upper-level kernel
bool coarse_batch_oversubscribe();       // false under TL_COARSE_BATCH_WG: launches fit at once
hipError_t launch_gather_ctrl(const BatchEntry* B, int n, Ctrl* out, hipStream_t stream);
// Band Cholesky factors of every set's relaxation region (overlap ov) into
// band (band_set_doubles(E + 2 ov) doubles per set).
hipError_t launch_band_factor(const Geo& g, int ov, const float* ea, const uint8_t* mask,
                              double* band, hipStream_t stream);
hipError_t launch_group1(const Geo& g, const float* ea, const uint8_t* mask, double* g1,
                         hipStream_t stream);
hipError_t launch_init_state(const Geo& g, const uint8_t* mask, const double2* u_fixed,
                             const double2* u_user, int warm, double2* u0,
                             double2* u1, void* d0, void* d1, bool mixed, double* a,
                             unsigned* flags, Ctrl* ctrl, hipStream_t stream);
hipError_t launch_copy_out(const Geo& g, const double2* u_pad, double2* u_user,
                           hipStream_t stream);
hipError_t launch_copy_delta(bool mixed, const Geo& g, const void* d_pad, double2* out,
                             hipStream_t stream);
// r = f - K u (unpadded f, u, r), and sums for R1, R2 (relative to the
// constrained right-hand side f - K_fc u_c, u_c = ufix or 0) and the energy.
hipError_t launch_residual(const Geo& g, const float* ea, const uint8_t* mask,
                           const double2* f, const double2* u, const double2* ufix, double2* r,
                           double* partials, double* out5, hipStream_t stream);
size_t residual_partials(const Geo& g);
// Pad and copy the lattice description; stats[0] += non-finite or negative
// EA count, stats[1] += clamped node count, stats[2] += free nodes whose own
// 2 x 2 stiffness block is singular.
hipError_t launch_pad_copy_stats(const Geo& g, const float* ea_user, const uint8_t* fixed_user,
                                 int ea_default, int fixed_default, float* ea, uint8_t* mask,
                                 int* stats, hipStream_t stream);

}  // namespace tl
