// HIP kernels of the hierarchical lattice solver (gfx950).
//
// One outer iteration of the method (Xu, Liu, Dong, section 2) is three
// launches:
//   k_tile    one workgroup per set (E x E node tile): applies the previous
//             upper-level correction (Eq. 3) to the tile and a one-node halo,
//             forms the float64 residual f - K u with the matrix-free rod
//             stencil, relaxes the set with its neighbours held fixed
//             (Eq. 11-13; preconditioned CG sweeps in LDS), and accumulates
//             the set's rows of the upper-level matrix for the relaxation
//             modes (Eq. 6, 13, 14) and its upper-level force (Eq. 7);
//   k_offdiag one workgroup per set: upper-level blocks between neighbouring
//             sets from the rods the set boundaries cut (Eq. 6);
//   k_coarse  persistent grid: global residual test (Eq. 19), then the
//             upper-level system (Eq. 8) by block-Jacobi PCG.
// Plus create-time, set-up and certification kernels.
#include "tl_internal.h"

#include <math.h>
#include <stdlib.h>

#include <algorithm>
#include <type_traits>

namespace tl {

namespace {

constexpr double kS3 = 0.86602540378443864676;   // sqrt(3)/2, y-step of a lattice row

__device__ __forceinline__ size_t pidx(const Geo& g, int i, int j) {
  return (size_t)(j + 1) * g.pitch + (size_t)(i + LPAD);
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous run of tiles so that halo rows shared by neighbouring tiles
// stay in one L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  constexpr int X = 8;
  const int xcd = b % X, k = b / X, per = nb / X, rem = nb % X;
  return xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

// Normalised coordinates of node (i, j) about the centre of its set tile
// [i0, i0 + tw) x [j0, j0 + th): xi = (x - xc) / (E/2), eta = (y - yc) / (E/2)
// with x = i + j/2, y = j*sqrt(3)/2 (representative node = tile centroid).
__device__ __forceinline__ void set_coords(int i, int j, int i0, int j0, int tw, int th,
                                           double inv_hs, double& xi, double& eta) {
  const double ic = i0 + 0.5 * (tw - 1), jc = j0 + 0.5 * (th - 1);
  xi = ((i - ic) + 0.5 * (j - jc)) * inv_hs;
  eta = ((j - jc) * kS3) * inv_hs;
}

// Wave sums with DPP lane moves (VALU operand modifiers, no LDS traffic):
// two quad exchanges, the half-row and row mirrors give every lane its
// 16-lane row sum, then the two row broadcasts carry the row sums to lane 63,
// whose value every lane reads.  All 64 lanes must be active (every call
// site is workgroup-uniform and every block is a whole number of waves).
// The order of the additions is fixed, so every wave adds the same way.
//
// The moves leave lanes outside their row mask undefined (no old value to
// set up first): those lanes' sums are never read, since every row mask
// holds row 3 and only lane 63 is.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, ROWS, 0xF, true));
}
__device__ __forceinline__ double lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// Lane l's value, l uniform across the wave.
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T v) {
  v += dpp_move<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);        // row_half_mirror
  v += dpp_move<0x140>(v);        // row_mirror
  v += dpp_move<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return lane63(v);
}
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }
__device__ __forceinline__ float wave_sum(float v) { return wave_sum_dpp(v); }
// Wave maximum, same lane moves; rows a broadcast skips keep their own value.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_move_keep(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move_keep<0xB1>(v));
  v = fmax(v, dpp_move_keep<0x4E>(v));
  v = fmax(v, dpp_move_keep<0x141>(v));
  v = fmax(v, dpp_move_keep<0x140>(v));
  v = fmax(v, dpp_move_keep<0x142, 0xA>(v));
  v = fmax(v, dpp_move_keep<0x143, 0xC>(v));
  return lane63(v);
}

// Wave sums of V values at once (V a power of two, at most 64) with about V
// shuffles instead of 6V: at each halving step a lane keeps half of the
// values it still holds and adds the partner's copy of that half, so after
// the six steps lane l holds the wave total of value l >> (6 - log2 V).
// Lanes that end with the same value hold the same bits.
//
// One halving step at lane offset O with H values still held; every index
// is a compile-time constant, so v stays in registers.
template <int V, int H, int O>
__device__ __forceinline__ void wave_sums_step(double (&v)[V], int lane) {
  if constexpr (H > 1) {
    constexpr int h = H / 2;
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int j = 0; j < h; ++j) {
      const double send = up ? v[j] : v[j + h];
      const double keep = up ? v[j + h] : v[j];
      v[j] = keep + __shfl_xor(send, O, 64);
    }
    if constexpr (O > 1) wave_sums_step<V, h, O / 2>(v, lane);
  } else {
    v[0] += __shfl_xor(v[0], O, 64);
    if constexpr (O > 1) wave_sums_step<V, 1, O / 2>(v, lane);
  }
}

template <int V>
__device__ __forceinline__ double wave_sums(double (&v)[V]) {
  static_assert(V >= 1 && V <= 64 && (V & (V - 1)) == 0, "V must be a power of two <= 64");
  wave_sums_step<V, V, 32>(v, threadIdx.x & 63);
  return v[0];
}

template <int V>
__device__ __forceinline__ int wave_sums_index() {
  constexpr int lg = V >= 64 ? 6 : V >= 32 ? 5 : V >= 16 ? 4 : V >= 8 ? 3 : V >= 4 ? 2 : V >= 2 ? 1 : 0;
  return (threadIdx.x & 63) >> (6 - lg);
}

// Workgroup sum; every thread gets the same (bitwise) value.  `slot` holds
// one entry per wave and must not be reused before the next barrier.
template <int NW, typename T>
__device__ __forceinline__ T block_sum(T v, double* slot) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = (double)v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += slot[w];
  return (T)s;
}

// Workgroup sum as a float64: the wave sums in the partials' own precision
// (float32 in the float32 sweeps, where DPP moves fold into the adds), the
// waves' totals in float64.  Same slot rules as block_sum.
template <int NW, typename T>
__device__ __forceinline__ double block_sum_wide(T v, double* slot) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = (double)v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += slot[w];
  return s;
}

// Workgroup sum of two values with one barrier; `slot` holds 2 entries per
// wave and must not be reused before the next barrier.
template <int NW>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* slot) {
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    slot[2 * (threadIdx.x >> 6)] = a;
    slot[2 * (threadIdx.x >> 6) + 1] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    sa += slot[2 * w];
    sb += slot[2 * w + 1];
  }
  a = sa;
  b = sb;
}

template <typename T> __device__ __forceinline__ typename V2<T>::type mk2(T x, T y);
template <> __device__ __forceinline__ float2 mk2<float>(float x, float y) { return make_float2(x, y); }
template <> __device__ __forceinline__ double2 mk2<double>(double x, double y) { return make_double2(x, y); }

}  // namespace

// ---------------------------------------------------------------------------
// Exact local solve (section 2.2 end: the local stiffness matrices do not
// change, so each is factored once and the factor reused).  A set's
// relaxation region of rw x rh nodes has n = 2 rw rh DOFs in row-major node
// order, x before y; a node's rods reach at most rw nodes ahead, so k^Inner
// is a band matrix of lower bandwidth b = 2 rw + 1.  Clamped DOFs become
// identity rows and columns (their residual is zero), so every region has a
// positive definite matrix of the same shape.  The factor L (k^Inner = L L^T)
// is stored column by column, BS doubles a column: 1/L_jj, then L_{j+1..j+b, j}.
// ---------------------------------------------------------------------------
namespace {

struct BandRegion {
  int ri0, rj0, rw, rh, n, b;
};

__device__ __forceinline__ BandRegion band_region(const Geo& g, int ov, int s) {
  const int E = g.E, I = s % g.mx, J = s / g.mx;
  const int i0 = I * E, j0 = J * E;
  const int tw = min(E, g.nx - i0), th = min(E, g.ny - j0);
  BandRegion r;
  r.ri0 = max(i0 - ov, 0);
  r.rj0 = max(j0 - ov, 0);
  r.rw = min(i0 + tw + ov, g.nx) - r.ri0;
  r.rh = min(j0 + th + ov, g.ny) - r.rj0;
  r.n = 2 * r.rw * r.rh;
  r.b = 2 * r.rw + 1;
  return r;
}

// Entry (k + d, k), 0 <= d <= b, of the region's k^Inner (identity on clamped
// DOFs; an identity column past the last DOF).
__device__ double band_entry(const Geo& g, const float* __restrict__ ea,
                             const uint8_t* __restrict__ mask, const BandRegion& br, int k, int d) {
  if (k >= br.n) return d == 0 ? 1.0 : 0.0;
  const int node = k >> 1, c = k & 1;
  const int li = node % br.rw, lj = node / br.rw;
  const size_t plane = (size_t)(g.ny + 2) * g.pitch;
  const size_t p = pidx(g, br.ri0 + li, br.rj0 + lj);
  if (mask[p]) return d == 0 ? 1.0 : 0.0;
  if (d == 0 || (d == 1 && c == 0)) {
    // the node's own 2x2 block: sum over its six rods of k n n^T
    const double ka = (double)ea[p] + (double)ea[p - 1];
    const double kb = (double)ea[plane + p] + (double)ea[plane + p - g.pitch];
    const double kc = (double)ea[2 * plane + p] + (double)ea[2 * plane + p - g.pitch + 1];
    if (d == 1) return 0.5 * kS3 * (kb - kc);
    return c == 0 ? ka + 0.25 * (kb + kc) : 0.75 * (kb + kc);
  }
  const int r = k + d;
  if (r >= br.n) return 0.0;
  const int m = r >> 1, c2 = r & 1, delta = m - node;
  // the forward neighbour at that DOF: east (+1), north-west (+rw - 1), north (+rw)
  double kr, nx_, ny_;
  int mi, mj;
  if (delta == 1 && li + 1 < br.rw) {
    kr = ea[p]; nx_ = 1.0; ny_ = 0.0; mi = li + 1; mj = lj;
  } else if (delta == br.rw - 1 && li > 0 && lj + 1 < br.rh) {
    kr = ea[2 * plane + p]; nx_ = -0.5; ny_ = kS3; mi = li - 1; mj = lj + 1;
  } else if (delta == br.rw && lj + 1 < br.rh) {
    kr = ea[plane + p]; nx_ = 0.5; ny_ = kS3; mi = li; mj = lj + 1;
  } else {
    return 0.0;
  }
  if (mask[pidx(g, br.ri0 + mi, br.rj0 + mj)]) return 0.0;
  return -kr * (c2 == 0 ? nx_ : ny_) * (c == 0 ? nx_ : ny_);
}

}  // namespace

// One workgroup per set: band Cholesky of its region's k^Inner, right-looking,
// with the b + 1 columns still being updated in an LDS ring (dynamic LDS of
// (b_max + 1) BS doubles); each column leaves the ring final and the next
// enters assembled.  A retiring column j is written to the column copy, and
// its entries L[j+d][j] to the row copy as entry d of row j + d; row j's
// entries before column 0 or past the band are zeros.
__global__ __launch_bounds__(256) void k_band_factor(Geo g, int ov, const float* __restrict__ ea,
                                                     const uint8_t* __restrict__ mask,
                                                     double* __restrict__ band) {
  extern __shared__ double ring[];
  const int s = blockIdx.x, t = threadIdx.x;
  const BandRegion br = band_region(g, ov, s);
  const int R = g.E + 2 * ov, BS = band_bs(R);
  const int n = br.n, b = br.b, nr = b + 1;
  double* out = band + (size_t)s * band_set_doubles(R);
  double* rows = out + band_copy_doubles(R);   // row r at (n - 1 - r) BS
  for (int e = t; e < nr * BS; e += 256) {
    const int col = e / BS, d = e % BS;
    ring[e] = d <= b ? band_entry(g, ea, mask, br, col, d) : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double* cj = ring + (size_t)(j % nr) * BS;
    const double ljj = sqrt(cj[0]);
    __syncthreads();   // every thread has read the pivot
    for (int d = 1 + t; d <= b; d += 256) cj[d] /= ljj;
    __syncthreads();
    // A[j+a+e][j+a] -= L[j+a+e][j] L[j+a][j], 1 <= a <= b, 0 <= e <= b - a
    for (int q = t; q < b * nr; q += 256) {
      const int a = 1 + q / nr, e = q % nr;
      if (e <= b - a) ring[(size_t)((j + a) % nr) * BS + e] -= cj[a + e] * cj[a];
    }
    __syncthreads();
    // retire column j; column j + b + 1 takes its slot
    for (int d = t; d < BS; d += 256) {
      const double lv = d == 0 ? 1.0 / ljj : (d <= b ? cj[d] : 0.0);
      out[(size_t)j * BS + d] = lv;
      if (d <= b && j + d < n) rows[(size_t)(n - 1 - j - d) * BS + d] = lv;
      if (d > min(j, b)) rows[(size_t)(n - 1 - j) * BS + d] = 0.0;
      cj[d] = d <= b ? band_entry(g, ea, mask, br, j + nr, d) : 0.0;
    }
    __syncthreads();
  }
}

// The six rods' neighbour terms of k^Inner times the node buffer at cell c
// (row pitch W), subtracted from (qx, qy).  In float32 opposite rods, which
// pull along the same unit vector, have their two axial terms summed before
// they are resolved into x and y: rods north and south along n1 = (1/2,
// sqrt3/2), north-west and south-east along n2 = (-1/2, sqrt3/2), with
// 2 n.p = +-p.x + sqrt3 p.y; east and west rods act on x alone.
template <typename T, int W, typename T2>
__device__ __forceinline__ void rod_neighbours(const T2* sp, const int c, const float* kq, T& qx,
                                               T& qy) {
  if constexpr (sizeof(T) == 8) {
    // (float64: one rod at a time, which holds fewer registers; summing the
    //  pairs first made the 32 x 32 tile spill 92 bytes per lane, not 36)
    T2 pb;
    T s;
    pb = sp[c + 1];     s = (T)kq[0] * pb.x;                                qx -= s;
    pb = sp[c - 1];     s = (T)kq[3] * pb.x;                                qx -= s;
    pb = sp[c + W];     s = (T)kq[1] * ((T)0.5 * pb.x + (T)kS3 * pb.y);   qx -= (T)0.5 * s; qy -= (T)kS3 * s;
    pb = sp[c - W];     s = (T)kq[4] * ((T)0.5 * pb.x + (T)kS3 * pb.y);   qx -= (T)0.5 * s; qy -= (T)kS3 * s;
    pb = sp[c + W - 1]; s = (T)kq[2] * ((T)-0.5 * pb.x + (T)kS3 * pb.y);  qx += (T)0.5 * s; qy -= (T)kS3 * s;
    pb = sp[c - W + 1]; s = (T)kq[5] * ((T)-0.5 * pb.x + (T)kS3 * pb.y);  qx += (T)0.5 * s; qy -= (T)kS3 * s;
    return;
  }
  constexpr T r3 = (T)(2.0 * kS3);
  const T2 pe = sp[c + 1], pw = sp[c - 1], pn = sp[c + W], ps = sp[c - W];
  const T2 pnw = sp[c + W - 1], pse = sp[c - W + 1];
  qx -= (T)kq[0] * pe.x + (T)kq[3] * pw.x;
  const T s1 = (T)kq[1] * (pn.x + r3 * pn.y) + (T)kq[4] * (ps.x + r3 * ps.y);     // 2 k n1.p
  const T s2 = (T)kq[2] * (r3 * pnw.y - pnw.x) + (T)kq[5] * (r3 * pse.y - pse.x);  // 2 k n2.p
  qx += (T)0.25 * (s2 - s1);
  qy -= (T)(0.5 * kS3) * (s1 + s2);
}

// alpha and beta of the relaxation sweeps from their float64 sums: a float64
// quotient in the float64 form; in the float32 form, which rounds them to
// float32 anyway, the sums rounded to float32 and the numerator times the
// hardware reciprocal of the denominator (within a few units of 2^-24).
template <typename T>
__device__ __forceinline__ T sweep_ratio(double num, double den) {
  if constexpr (sizeof(T) == 4) return (float)num * __builtin_amdgcn_rcpf((float)den);
  else return num / den;
}

// ---------------------------------------------------------------------------
// Tile kernel: update + residual + local relaxation + set's upper-level rows.
// ---------------------------------------------------------------------------
//
// OV is the overlap of the relaxation region (section 2.2 end): the set's
// tile widened by OV nodes on every side, clipped to the lattice.  The update
// and the residual cover the region (plus a one-node ring for the stencil),
// the relaxation solves on the region's free DOFs with everything outside it
// held fixed, and the increment, the stop-test norms and the upper-level rows
// use the set's own nodes only.  OV = 0 is the plain set.
template <typename T, int E, int NT, int OV>
__device__ __forceinline__ void tile_body(const Geo& g, const float* __restrict__ ea,
                                          const uint8_t* __restrict__ mask, const TileArgs& A,
                                          const int tile) {
  using T2 = typename V2<T>::type;
  constexpr int R = E + 2 * OV;                 // region edge before clipping
  constexpr int NPT = (R * R + NT - 1) / NT;
  constexpr int W = R + 2;
  constexpr int NW = NT / 64;
  static_assert(OV + 1 <= E, "the region's ring must stay within the neighbouring sets");
  __shared__ double2 su[W * W];                 // u over region + ring, then T2 p / delta
  __shared__ double sa[9][Q];                   // coefficients of the 3x3 set neighbourhood
  __shared__ double sred[3][NW];
  __shared__ double sacc[NW][KROW + 3];
  __shared__ double sfin[11];
  // The region's float64 residual waits in LDS, not in registers, for the
  // relaxation's start and the upper-level rows, when it fits beside the
  // node buffer: with 64 x 64 sets (four or more nodes per thread), and in
  // the float64 form with 32 x 32 sets, whose tiles are held to 128
  // registers so that two share a CU (1024^2: spill 112 -> 68 bytes per
  // lane, launch 153 -> 148 us; the float32 tile gained nothing).
  constexpr bool kResidLds = (E >= 64 || (E == 32 && sizeof(T) == 8)) &&
                             (W * W + R * R) * 16 + 8192 <= 160 * 1024;
  constexpr bool kLoadAhead = E >= 64;   // residual loads run ahead of the arithmetic
  __shared__ double2 sres[kResidLds ? R * R : 1];
  T2* sp = reinterpret_cast<T2*>(su);

  if (A.ctrl->done) return;
  const int kit = A.ctrl->k;
  const double2* u_in = (kit & 1) ? A.u1 : A.u0;
  double2* u_out = (kit & 1) ? A.u0 : A.u1;
  const void* d_in_v = (kit & 1) ? A.d1 : A.d0;
  void* d_out_v = (kit & 1) ? A.d0 : A.d1;
  const int I = tile % g.mx, J = tile / g.mx;
  const int i0 = I * E, j0 = J * E;
  const int tw = min(E, g.nx - i0), th = min(E, g.ny - j0);
  const int ri0 = max(i0 - OV, 0), rj0 = max(j0 - OV, 0);      // relaxation region
  const int rw = min(i0 + tw + OV, g.nx) - ri0, rh = min(j0 + th + OV, g.ny) - rj0;
  const int t = threadIdx.x;
  const size_t plane = (size_t)(g.ny + 2) * g.pitch;
  const double inv_hs = 2.0 / E;

  if (t < 81) {
    const int s = t / Q, m = t % Q;
    const int I2 = I + (s % 3) - 1, J2 = J + (s / 3) - 1;
    sa[s][m] = (I2 >= 0 && I2 < g.mx && J2 >= 0 && J2 < g.my)
                   ? A.a[(size_t)(J2 * g.mx + I2) * Q + m] : 0.0;
  }
  __syncthreads();

  // 1. u_new = u_old + sum_m a_m u_hat_m (Eq. 3) on the region and its ring.
  //    All loads of a thread's nodes are issued before any is used, so the
  //    phase costs one memory latency instead of one per node.
  {
    constexpr int RIT = (W * W + NT - 1) / NT;
    const T2* din = reinterpret_cast<const T2*>(d_in_v);
    const int ew = rw + 2, rn = (rw + 2) * (rh + 2);
    double2 ul[RIT];
    T2 dl[RIT];
    uint8_t ml[RIT];
#pragma unroll
    for (int k = 0; k < RIT; ++k) {
      const int idx = t + k * NT;
      ml[k] = 1;
      ul[k] = make_double2(0.0, 0.0);
      dl[k] = mk2<T>((T)0, (T)0);
      if (idx < rn) {
        const size_t p = pidx(g, ri0 - 1 + idx % ew, rj0 - 1 + idx / ew);
        ul[k] = u_in[p];
        ml[k] = mask[p];
        dl[k] = din[p];
      }
    }
#pragma unroll
    for (int k = 0; k < RIT; ++k) {
      const int idx = t + k * NT;
      if (idx >= rn) continue;
      const int ri = idx % ew, rj = idx / ew;
      const int gi = ri0 - 1 + ri, gj = rj0 - 1 + rj;
      double2 u = ul[k];
      if (!ml[k]) {            // a lattice node (the padding ring is masked)
        const int dI = gi / E - I, dJ = gj / E - J;
        const int oi0 = (I + dI) * E, oj0 = (J + dJ) * E;
        double xi, eta;
        set_coords(gi, gj, oi0, oj0, min(E, g.nx - oi0), min(E, g.ny - oj0), inv_hs, xi, eta);
        const double* c = sa[(dJ + 1) * 3 + (dI + 1)];
        const double w = c[6] + c[7] * xi + c[8] * eta;
        u.x += c[0] + c[2] * xi + c[3] * eta + w * (double)dl[k].x;
        u.y += c[1] + c[4] * xi + c[5] * eta + w * (double)dl[k].y;
      }
      su[rj * W + ri] = u;
      if (gi >= i0 && gi < i0 + tw && gj >= j0 && gj < j0 + th) u_out[pidx(g, gi, gj)] = u;
    }
  }
  __syncthreads();

  // 2. residual r = f - K u (float64) and the per-node relaxation operator.
  float kk[NPT][6];
  double2 r[NPT];
  T idet[NPT];                       // 1 / det of the node's 2x2 diagonal block
  bool act[NPT], own[NPT];
  double part[10];   // P1..P6, sum|r|, sum r^2, sum|f|, sum f^2
#pragma unroll
  for (int v = 0; v < 10; ++v) part[v] = 0.0;
  double rmax = 0.0;
  double2 fl[NPT];
  // all of the thread's loads first (one memory latency), then the arithmetic
  auto load_node = [&](const int k) {
    const int n = t + k * NT, li = n % R, lj = n / R;
    act[k] = false;
    own[k] = false;
    fl[k] = make_double2(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < 6; ++b) kk[k][b] = 0.f;
    if (n < R * R && li < rw && lj < rh) {
      const int gi = ri0 + li, gj = rj0 + lj;
      const size_t p = pidx(g, gi, gj);
      act[k] = mask[p] == 0;
      own[k] = act[k] && gi >= i0 && gi < i0 + tw && gj >= j0 && gj < j0 + th;
      kk[k][0] = ea[p];
      kk[k][1] = ea[plane + p];
      kk[k][2] = ea[2 * plane + p];
      kk[k][3] = ea[p - 1];
      kk[k][4] = ea[plane + p - g.pitch];
      kk[k][5] = ea[2 * plane + p - g.pitch + 1];
      fl[k] = A.f[(size_t)gj * g.nx + gi];
    }
  };
  // With 64 x 64 sets the loads of all of a thread's nodes do not fit in
  // registers beside the arithmetic: the loads then run kAhead nodes ahead of
  // the arithmetic (node k + kAhead's issued before node k's arithmetic),
  // fenced so the scheduler keeps that order: two with 256 registers per
  // thread (at most 512 threads), one with 128.
  if constexpr (!kLoadAhead) {
#pragma unroll
    for (int k = 0; k < NPT; ++k) load_node(k);
  }
  constexpr int kAhead = NT <= 512 ? 2 : 1;
  if constexpr (kLoadAhead) {
#pragma unroll
    for (int k = 0; k < kAhead && k < NPT; ++k) load_node(k);
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    if constexpr (kLoadAhead) {
      __builtin_amdgcn_sched_barrier(0);
      if (k + kAhead < NPT) load_node(k + kAhead);
    }
    const int n = t + k * NT, li = n % R, lj = n / R;
    r[k] = make_double2(0.0, 0.0);
    idet[k] = (T)0;
    if (!act[k]) continue;
    const int gi = ri0 + li, gj = rj0 + lj;
    const size_t p = pidx(g, gi, gj);
    const int c = (lj + 1) * W + (li + 1);
    const double2 ua = su[c];
    double kx = 0.0, ky = 0.0;
    auto rod = [&](float kb, double nx_, double ny_, double2 ub) {
      const double s = (double)kb * (nx_ * (ua.x - ub.x) + ny_ * (ua.y - ub.y));
      kx += s * nx_;
      ky += s * ny_;
    };
    rod(kk[k][0], 1.0, 0.0, su[c + 1]);
    rod(kk[k][1], 0.5, kS3, su[c + W]);
    rod(kk[k][2], -0.5, kS3, su[c + W - 1]);
    rod(kk[k][3], 1.0, 0.0, su[c - 1]);
    rod(kk[k][4], 0.5, kS3, su[c - W]);
    rod(kk[k][5], -0.5, kS3, su[c - W + 1]);
    double2 fv = fl[k];
    const double rx = fv.x - kx, ry = fv.y - ky;
    if (A.rhs_mode) {
      // right-hand side of the constrained system: f - K_fc u_c, i.e. the
      // load plus the pull of every rod that ends on a clamped node
      const int cb[6] = {c + 1, c - 1, c + W, c - W, c + W - 1, c - W + 1};
      const long pb[6] = {1, -1, g.pitch, -(long)g.pitch, (long)g.pitch - 1, -(long)g.pitch + 1};
      const double nbx[6] = {1.0, 1.0, 0.5, 0.5, -0.5, -0.5};
      const double nby[6] = {0.0, 0.0, kS3, kS3, kS3, kS3};
      const int kb[6] = {0, 3, 1, 4, 2, 5};
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        if (!mask[(long)p + pb[b]]) continue;
        const double2 ub = su[cb[b]];
        const double sv = (double)kk[k][kb[b]] * (nbx[b] * ub.x + nby[b] * ub.y);
        fv.x += sv * nbx[b];
        fv.y += sv * nby[b];
      }
    }
    r[k] = make_double2(rx, ry);
    if constexpr (kResidLds) sres[t + k * NT] = r[k];
    rmax = fmax(rmax, fmax(fabs(rx), fabs(ry)));
    if (own[k]) {
      double xi, eta;
      set_coords(gi, gj, i0, j0, tw, th, inv_hs, xi, eta);
      part[0] += rx;
      part[1] += ry;
      part[2] += xi * rx;
      part[3] += eta * rx;
      part[4] += xi * ry;
      part[5] += eta * ry;
      part[6] += fabs(rx) + fabs(ry);
      part[7] += rx * rx + ry * ry;
      part[8] += fabs(fv.x) + fabs(fv.y);
      part[9] += fv.x * fv.x + fv.y * fv.y;
    }
    // diagonal 2x2 block of k^Inner: sum over all six rods of k n n^T
    const double ka = (double)kk[k][0] + kk[k][3];
    const double kb = (double)kk[k][1] + kk[k][4];
    const double kc = (double)kk[k][2] + kk[k][5];
    const double Dxx = ka + 0.25 * (kb + kc), Dyy = 0.75 * (kb + kc), Dxy = 0.5 * kS3 * (kb - kc);
    const double det = Dxx * Dyy - Dxy * Dxy;
    idet[k] = (T)(1.0 / det);
  }
  // workgroup reduction of the 10 partials and the max |r|
  {
    // (the many-value wave sums pay off where their registers fit: up to
    //  three nodes per thread, or 256 registers per thread with at most 512
    //  threads; with 64 x 64 sets in 1024 threads they spill)
    if constexpr (NPT <= 3 || NT <= 512) {
      double p16[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) p16[v] = v < 10 ? part[v] : 0.0;
      const double ps = wave_sums<16>(p16);
      const int v = wave_sums_index<16>();
      if ((t & 3) == 0 && v < 10) sacc[t >> 6][v] = ps;
    } else {
#pragma unroll
      for (int v = 0; v < 10; ++v) part[v] = wave_sum(part[v]);
      if ((t & 63) == 0) {
#pragma unroll
        for (int v = 0; v < 10; ++v) sacc[t >> 6][v] = part[v];
      }
    }
    rmax = wave_max(rmax);
    if ((t & 63) == 0) sacc[t >> 6][10] = rmax;
    __syncthreads();   // also: every read of su as u is done
    if (t < 11) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s = t == 10 ? fmax(s, sacc[w][10]) : s + sacc[w][t];
      sfin[t] = s;
    }
    // zero the relaxation buffer (region, its ring and inactive nodes)
    for (int idx = t; idx < W * W; idx += NT) sp[idx] = mk2<T>((T)0, (T)0);
    __syncthreads();
  }
  if (t < 6) A.force[(size_t)tile * Q + t] = sfin[t];
  if (t >= 6 && t < 10) A.nrm[(size_t)tile * NRM + (t - 6)] = sfin[t];

  // 3. local relaxation: k^Inner delta = r on the region's free DOFs, the
  //    rest held fixed (Eq. 12 minus k^Inner u_old), by block-Jacobi PCG.
  //    Float32 form: r is scaled by 2^-e (e from max|r|) before rounding.
  const double rm = sfin[10];
  const double scl = (sizeof(T) == 4 && rm > 0.0 && isfinite(rm)) ? ldexp(1.0, -ilogb(rm)) : 1.0;
  // The sweep comes in two forms with the same iterates in exact arithmetic.
  // With float32 sets of up to 32 x 32 nodes it exchanges z through LDS in
  // the barrier interval of r.z (two barriers a sweep); in float64 and with
  // 64 x 64 sets that form holds more registers and spills, so there the
  // direction p is exchanged (three barriers a sweep, no spill added).
  constexpr bool kTwoBarrier = sizeof(T) == 4 && E <= 32;
  T2 x[NPT];
  bool exact = false;
  if constexpr (sizeof(T) == 8 && E <= 32) {   // the float64 form with sets up to 32 x 32
    if (A.band) {
      // Exact local solve (section 2.2 end): k^Inner delta = r on the
      // region with the set's band factor, L y = r, then L^T delta = y.
      // Both are one kind of pass: step j takes the final v[j] (times the
      // stored 1/L_jj) and subtracts its multiples from v[j+1 .. j+b], with
      // the factor's columns (forward) or its rows in descending order
      // (backward, positions mirrored).  The residual goes to the node buffer
      // in DOF order.  Wave 0 runs the steps with v in registers: positions
      // 64k .. 64k + 191 of the current block k, position p in lane p % 64,
      // and the next pivot read from its lane before the step's updates, so
      // that one multiply-add per step depends on the last.  The other waves
      // stage the next BAND_CH factor columns into LDS meanwhile.
      exact = true;
      extern __shared__ double band_lds[];
      constexpr int BS = band_bs(R);
      const int n = 2 * rw * rh, b = 2 * rw + 1;
      const double* Lg = A.band + (size_t)tile * A.band_stride;
      double* v = reinterpret_cast<double*>(su);
      auto residual_at = [&](const int k) -> double2 {
        return kResidLds ? sres[t + k * NT] : r[k];
      };
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int nn = t + k * NT, li = nn % R, lj = nn / R;
        if (nn < R * R && li < rw && lj < rh) {
          const double2 rk = act[k] ? residual_at(k) : make_double2(0.0, 0.0);
          const int dof = 2 * (lj * rw + li);
          v[dof] = rk.x;
          v[dof + 1] = rk.y;
        }
      }
      const int nch = (n + BAND_CH - 1) / BAND_CH;
      const int wave = t >> 6, lane = t & 63;
      double* buf0 = band_lds;
      double* buf1 = band_lds + BAND_CH * BS;
      // a chunk goes through registers: every load is issued before the
      // first LDS write waits for its data
      auto load_chunk = [&](auto nth_c, const double* Lc, const int c, double* buf, const int t0) {
        constexpr int nth = decltype(nth_c)::value;
        const int cnt = min(BAND_CH, n - c * BAND_CH) * (BS / 2);
        const double2* src = reinterpret_cast<const double2*>(Lc + (size_t)c * BAND_CH * BS);
        double2* dst = reinterpret_cast<double2*>(buf);
        for (int e0 = t0; e0 < cnt; e0 += 4 * nth) {
          const bool g1 = e0 + nth < cnt, g2 = e0 + 2 * nth < cnt, g3 = e0 + 3 * nth < cnt;
          const double2 a = src[e0];
          const double2 bb = g1 ? src[e0 + nth] : a;
          const double2 cc = g2 ? src[e0 + 2 * nth] : a;
          const double2 dd = g3 ? src[e0 + 3 * nth] : a;
          dst[e0] = a;
          if (g1) dst[e0 + nth] = bb;
          if (g2) dst[e0 + 2 * nth] = cc;
          if (g3) dst[e0 + 3 * nth] = dd;
        }
      };
      using AllThreads = std::integral_constant<int, NT>;
      using Loaders = std::integral_constant<int, NT - 64>;
      auto pass = [&](const double* Lc, const bool mirror) {
        auto at = [&](const int p) { return mirror ? n - 1 - p : p; };
        load_chunk(AllThreads{}, Lc, 0, buf0, t);
        __syncthreads();   // chunk 0, and v complete
        double w0 = 0.0, w1 = 0.0, w2 = 0.0, piv = 0.0, yprev = 0.0, lprev = 0.0;
        if (wave == 0) {
          w0 = lane < n ? v[at(lane)] : 0.0;
          w1 = lane + 64 < n ? v[at(lane + 64)] : 0.0;
          w2 = lane + 128 < n ? v[at(lane + 128)] : 0.0;
          piv = lane_value(w0, 0);
        }
        for (int c = 0; c < nch; ++c) {
          const double* cur = (c & 1) ? buf1 : buf0;
          if (wave != 0) {
            if (c + 1 < nch) load_chunk(Loaders{}, Lc, c + 1, (c & 1) ? buf0 : buf1, t - 64);
          } else {
            const int jend = min(BAND_CH, n - c * BAND_CH);
            // Step jj needs entries lane - jj, lane + 64 - jj and lane + 128 - jj
            // of column jj: one per-lane address, advanced by BS - 1 doubles a
            // step, serves all three (the buffers are padded so that reads
            // of entries past the band stay in LDS; their lanes do not use
            // them).  The next step's reads are issued before this step's
            // arithmetic, and the block's last step, whose next pivot is in
            // the window's second register, is peeled.
            const double* pl = cur + lane;
            int dl = lane;   // lane - jj
            const int b1 = b - 64, b2 = b - 128;
            double c0 = cur[0], c1 = cur[1], l0 = pl[0], l1 = pl[64], l2 = pl[128];
            auto step = [&](const int jj, auto last_c) {
              constexpr bool last = decltype(last_c)::value;
              double nc0 = 0.0, nc1 = 0.0, nl0 = 0.0, nl1 = 0.0, nl2 = 0.0;
              if constexpr (!last) {
                const double* ncol = cur + (jj + 1) * BS;
                const double* np = pl + (BS - 1);
                nc0 = ncol[0];
                nc1 = ncol[1];
                nl0 = np[0];
                nl1 = np[64];
                nl2 = np[128];
              }
              __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the arithmetic
              // piv is v[j] before step j - 1 subtracted its multiple: y_j =
              // (piv - L[j][j-1] y_{j-1}) / L_jj, one multiply-add after y_{j-1}
              const double yj = fma(-(lprev * c0), yprev, piv * c0);
              piv = lane_value(last ? w1 : w0, (jj + 1) & 63);
              lprev = c1;
              if (dl >= 1 && dl <= b) w0 = fma(-l0, yj, w0);
              if (dl == 0) w0 = yj;
              if (dl <= b1) w1 = fma(-l1, yj, w1);
              if (dl <= b2) w2 = fma(-l2, yj, w2);
              yprev = yj;
              c0 = nc0;
              c1 = nc1;
              l0 = nl0;
              l1 = nl1;
              l2 = nl2;
              pl += BS - 1;
              --dl;
            };
            const int jfull = min(jend, BAND_CH - 1);
            for (int jj = 0; jj < jfull; ++jj) step(jj, std::false_type{});
            if (jend == BAND_CH) step(BAND_CH - 1, std::true_type{});
            // positions 64c .. 64c + 63 are final: store them, move the window
            if (c * 64 + lane < n) v[at(c * 64 + lane)] = w0;
            w0 = w1;
            w1 = w2;
            w2 = (c + 3) * 64 + lane < n ? v[at((c + 3) * 64 + lane)] : 0.0;
          }
          __syncthreads();
        }
      };
      static_assert(BAND_CH == 64, "a chunk is one block of the register window");
      pass(Lg, false);
      pass(Lg + A.band_stride / 2, true);
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const int nn = t + k * NT, li = nn % R, lj = nn / R;
        x[k] = mk2<T>((T)0, (T)0);
        if (nn < R * R && li < rw && lj < rh && act[k]) {
          const int dof = 2 * (lj * rw + li);
          x[k] = mk2<T>((T)v[dof], (T)v[dof + 1]);
        }
      }
      __syncthreads();   // every read of the buffer as v is done
      for (int idx = t; idx < W * W; idx += NT) sp[idx] = mk2<T>((T)0, (T)0);
      __syncthreads();
    }
  }
  if (exact) {
    // (the increment is in x)
  } else if constexpr (kTwoBarrier) {
    // Per node only x, r, p, K p and 1/det B stay in registers across the
    // sweep's barriers (register pressure): the 2x2 diagonal block B is rebuilt
    // from the rod stiffnesses, and z = B^-1 r = adj(B) r / det B goes straight
    // to the LDS buffer.
    //
    // Two barriers per sweep.  The preconditioned residual z, not the search
    // direction, is exchanged through LDS, in the same barrier interval as the
    // partial sums of r.z; after that barrier beta is known, so the direction
    // p = z + beta p and its product K p = K z + beta K p (the recurrence of
    // the previous product) follow without a further exchange, and the second
    // barrier is the one of p.Kp.  In exact arithmetic these are the iterates
    // of plain PCG.
    T2 rr[NPT], pp[NPT], qq[NPT];
    auto precond = [&](const int k, const T2 rv) {
      const T ka = (T)kk[k][0] + (T)kk[k][3], kb = (T)kk[k][1] + (T)kk[k][4];
      const T kc = (T)kk[k][2] + (T)kk[k][5];
      const T Dxx = ka + (T)0.25 * (kb + kc), Dyy = (T)0.75 * (kb + kc);
      const T Dxy = (T)(0.5 * kS3) * (kb - kc);
      return mk2<T>(idet[k] * (Dyy * rv.x - Dxy * rv.y), idet[k] * (Dxx * rv.y - Dxy * rv.x));
    };
    // k^Inner applied to the buffer at active node k (own value za)
    auto apply_k = [&](const int k, const int c, const T2 za) {
      // (float64 form: the stiffnesses pass an empty asm so that each sweep
      //  converts them afresh instead of the compiler holding the residual
      //  step's conversions in registers across the relaxation)
      float kq[6];
  #pragma unroll
      for (int b = 0; b < 6; ++b) {
        kq[b] = kk[k][b];
        if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(kq[b]));
      }
      const T ka = (T)kq[0] + (T)kq[3], kb = (T)kq[1] + (T)kq[4];
      const T kc = (T)kq[2] + (T)kq[5];
      const T Dxx = ka + (T)0.25 * (kb + kc), Dyy = (T)0.75 * (kb + kc);
      const T Dxy = (T)(0.5 * kS3) * (kb - kc);
      T qx = Dxx * za.x + Dxy * za.y;
      T qy = Dxy * za.x + Dyy * za.y;
      rod_neighbours<T, W>(sp, c, kq, qx, qy);
      return mk2<T>(qx, qy);
    };
    auto cell = [&](const int k) { const int n = t + k * NT; return (n / R + 1) * W + (n % R + 1); };
    // z = B^-1 r into the buffer; returns this thread's part of r.z
    auto publish_z = [&]() {
      T part = (T)0;   // a thread's nodes summed in the sweep's precision
  #pragma unroll
      for (int k = 0; k < NPT; ++k) {
        const T2 z = precond(k, rr[k]);
        if (act[k]) sp[cell(k)] = z;
        part += rr[k].x * z.x + rr[k].y * z.y;
      }
      return part;
    };
    // p = z + beta p, K p = K z + beta K p; returns this thread's part of p.Kp
    auto next_direction = [&](const T beta) {
      T part = (T)0;
  #pragma unroll
      for (int k = 0; k < NPT; ++k) {
        if (!act[k]) { pp[k] = qq[k] = mk2<T>((T)0, (T)0); continue; }
        const int c = cell(k);
        const T2 z = sp[c];
        const T2 w = apply_k(k, c, z);
        pp[k].x = z.x + beta * pp[k].x;  pp[k].y = z.y + beta * pp[k].y;
        qq[k].x = w.x + beta * qq[k].x;  qq[k].y = w.y + beta * qq[k].y;
        part += pp[k].x * qq[k].x + pp[k].y * qq[k].y;
      }
      return part;
    };
  #pragma unroll
    for (int k = 0; k < NPT; ++k) {
      x[k] = mk2<T>((T)0, (T)0);
      pp[k] = qq[k] = mk2<T>((T)0, (T)0);
      const double2 rk = kResidLds ? (act[k] ? sres[t + k * NT] : make_double2(0.0, 0.0)) : r[k];
      rr[k] = mk2<T>((T)(rk.x * scl), (T)(rk.y * scl));
    }
    double rz = block_sum_wide<NW>(publish_z(), sred[0]);
    // The sweeps end early, uniformly across the workgroup, when the PCG has
    // nothing left to gain: p.Kp <= 0, or r.z has fallen below 2^-60 of its
    // start in float32 (2^-120 in float64), far past the precision's attainable
    // accuracy.  Past that point the recurrences of a small region run on
    // underflowing values, and in float32 they can diverge after a thousand or
    // so further sweeps.  The default sweep counts never reach the threshold.
    const double rz_stop = rz * (sizeof(T) == 4 ? 0x1p-60 : 0x1p-120);
    double pq = block_sum_wide<NW>(next_direction((T)0), sred[1]);
    for (int it = 0; it < A.inner_iters; ++it) {
      if (!(pq > 0.0)) break;
      const T alpha = sweep_ratio<T>(rz, pq);
  #pragma unroll
      for (int k = 0; k < NPT; ++k) {
        x[k].x += alpha * pp[k].x;  x[k].y += alpha * pp[k].y;
        rr[k].x -= alpha * qq[k].x; rr[k].y -= alpha * qq[k].y;
      }
      if (it + 1 == A.inner_iters) break;
      // (the buffer is free: every read of it as z came before the last p.Kp
      //  barrier; likewise the slots of each sum before the other's barrier)
      const double rzn = block_sum_wide<NW>(publish_z(), sred[0]);
      if (!(rzn > rz_stop)) break;
      const T beta = rz > 0.0 ? sweep_ratio<T>(rzn, rz) : (T)0;
      rz = rzn;
      pq = block_sum_wide<NW>(next_direction(beta), sred[1]);
    }

  } else {
    // Per node only x, r, p, K p and 1/det B stay in registers across the
    // sweep's barriers (register pressure): the 2x2 diagonal block B is rebuilt
    // from the rod stiffnesses, z = B^-1 r = adj(B) r / det B is formed once
    // per sweep and waits for the direction update in the K p slot.
    T2 rr[NPT], pp[NPT], qq[NPT];
    auto precond = [&](const int k, const T2 rv) {
      const T ka = (T)kk[k][0] + (T)kk[k][3], kb = (T)kk[k][1] + (T)kk[k][4];
      const T kc = (T)kk[k][2] + (T)kk[k][5];
      const T Dxx = ka + (T)0.25 * (kb + kc), Dyy = (T)0.75 * (kb + kc);
      const T Dxy = (T)(0.5 * kS3) * (kb - kc);
      return mk2<T>(idet[k] * (Dyy * rv.x - Dxy * rv.y), idet[k] * (Dxx * rv.y - Dxy * rv.x));
    };
    T rz_part = (T)0;   // a thread's nodes summed in the sweep's precision
  #pragma unroll
    for (int k = 0; k < NPT; ++k) {
      x[k] = mk2<T>((T)0, (T)0);
      const double2 rk = kResidLds ? (act[k] ? sres[t + k * NT] : make_double2(0.0, 0.0)) : r[k];
      rr[k] = mk2<T>((T)(rk.x * scl), (T)(rk.y * scl));
      pp[k] = precond(k, rr[k]);
      rz_part += rr[k].x * pp[k].x + rr[k].y * pp[k].y;
    }
    double rz = block_sum_wide<NW>(rz_part, sred[0]);
    // The sweeps end early, uniformly across the workgroup, when the PCG has
    // nothing left to gain: p.Kp <= 0, or r.z has fallen below 2^-60 of its
    // start in float32 (2^-120 in float64), far past the precision's attainable
    // accuracy.  Past that point the recurrences of a small region run on
    // underflowing values, and in float32 they can diverge after a thousand or
    // so further sweeps.  The default sweep counts never reach the threshold.
    const double rz_stop = rz * (sizeof(T) == 4 ? 0x1p-60 : 0x1p-120);
    for (int it = 0; it < A.inner_iters; ++it) {
  #pragma unroll
      for (int k = 0; k < NPT; ++k) {
        if (!act[k]) continue;
        const int n = t + k * NT;
        sp[(n / R + 1) * W + (n % R + 1)] = pp[k];
      }
      __syncthreads();
      T pq_part = (T)0;
  #pragma unroll
      for (int k = 0; k < NPT; ++k) {
        if (!act[k]) { qq[k] = mk2<T>((T)0, (T)0); continue; }
        const int n = t + k * NT;
        const int c = (n / R + 1) * W + (n % R + 1);
        const T2 pa = pp[k];
        // (float64 form: the stiffnesses pass an empty asm so that each sweep
        //  converts them afresh instead of the compiler holding the residual
        //  step's conversions in registers across the relaxation)
        float kq[6];
  #pragma unroll
        for (int b = 0; b < 6; ++b) {
          kq[b] = kk[k][b];
          if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(kq[b]));
        }
        const T ka = (T)kq[0] + (T)kq[3], kb = (T)kq[1] + (T)kq[4];
        const T kc = (T)kq[2] + (T)kq[5];
        const T Dxx = ka + (T)0.25 * (kb + kc), Dyy = (T)0.75 * (kb + kc);
        const T Dxy = (T)(0.5 * kS3) * (kb - kc);
        T qx = Dxx * pa.x + Dxy * pa.y;
        T qy = Dxy * pa.x + Dyy * pa.y;
        rod_neighbours<T, W>(sp, c, kq, qx, qy);
        qq[k] = mk2<T>(qx, qy);
        pq_part += pa.x * qx + pa.y * qy;
      }
      const double pq = block_sum_wide<NW>(pq_part, sred[1]);
      if (!(pq > 0.0)) break;
      const T alpha = sweep_ratio<T>(rz, pq);
      T rzn_part = (T)0;
  #pragma unroll
      for (int k = 0; k < NPT; ++k) {
        x[k].x += alpha * pp[k].x;  x[k].y += alpha * pp[k].y;
        rr[k].x -= alpha * qq[k].x; rr[k].y -= alpha * qq[k].y;
        qq[k] = precond(k, rr[k]);
        rzn_part += rr[k].x * qq[k].x + rr[k].y * qq[k].y;
      }
      const double rzn = block_sum_wide<NW>(rzn_part, sred[it & 1 ? 0 : 2]);
      const T beta = rz > 0.0 ? sweep_ratio<T>(rzn, rz) : (T)0;
      rz = rzn;
  #pragma unroll
      for (int k = 0; k < NPT; ++k) {
        pp[k].x = qq[k].x + beta * pp[k].x;
        pp[k].y = qq[k].y + beta * pp[k].y;
      }
      if (!(rz > rz_stop)) break;
    }

  }

  // 4. store the relaxation increment on the set's own nodes (mode 7 as
  //    stored, scaled in float32); the buffer keeps it on those nodes only.
  {
    T2* dout = reinterpret_cast<T2*>(d_out_v);
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int n = t + k * NT, li = n % R, lj = n / R;
      if (n < R * R && li < rw && lj < rh) {
        const int gi = ri0 + li, gj = rj0 + lj;
        const T2 d = own[k] ? x[k] : mk2<T>((T)0, (T)0);
        if (gi >= i0 && gi < i0 + tw && gj >= j0 && gj < j0 + th) dout[pidx(g, gi, gj)] = d;
        if (act[k]) sp[(lj + 1) * W + (li + 1)] = d;   // zero on the overlap nodes
      }
    }
  }
  __syncthreads();

  // 5. rows 7-9 of the set's diagonal upper-level block, K[m][l] =
  //    u_hat_m . k^Inner u_hat_l for l in {delta, xi*delta, eta*delta} (Eq. 6),
  //    and P_7..9 = u_hat_l . r (Eq. 7), all in float64.
  double acc[KROW + 3];
#pragma unroll
  for (int v = 0; v < KROW + 3; ++v) acc[v] = 0.0;
  const double dxi[6] = {inv_hs, -inv_hs, 0.5 * inv_hs, -0.5 * inv_hs, -0.5 * inv_hs, 0.5 * inv_hs};
  const double deta[6] = {0.0, 0.0, kS3 * inv_hs, -kS3 * inv_hs, kS3 * inv_hs, -kS3 * inv_hs};
  const double nvx[6] = {1.0, 1.0, 0.5, 0.5, -0.5, -0.5};
  const double nvy[6] = {0.0, 0.0, kS3, kS3, kS3, kS3};
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    if (!own[k]) continue;
    const int n = t + k * NT, li = n % R, lj = n / R;
    const int c = (lj + 1) * W + (li + 1);
    const int off[6] = {1, -1, W, -W, W - 1, -W + 1};
    const int kidx[6] = {0, 3, 1, 4, 2, 5};
    double xi, eta;
    set_coords(ri0 + li, rj0 + lj, i0, j0, tw, th, inv_hs, xi, eta);
    const double dax = (double)x[k].x, day = (double)x[k].y;
    // k^Inner applied rod by rod, each rod's diagonal part beside its
    // coupling to the neighbour.  The stiffnesses pass an empty asm first:
    // otherwise the compiler reuses the float64 conversions of the residual
    // step and keeps them live across the whole relaxation, which with many
    // nodes per thread spills them.
    float kf[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      kf[b] = kk[k][b];
      asm volatile("" : "+v"(kf[b]));
    }
    double w7x = 0.0, w7y = 0.0, w8x = 0.0, w8y = 0.0, w9x = 0.0, w9y = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      const T2 db = sp[c + off[b]];
      const double kr = (double)kf[kidx[b]];
      const double sa = kr * (nvx[b] * dax + nvy[b] * day);
      const double s7 = kr * (nvx[b] * (double)db.x + nvy[b] * (double)db.y);
      const double d7 = sa - s7;
      const double d8 = xi * sa - (xi + dxi[b]) * s7;
      const double d9 = eta * sa - (eta + deta[b]) * s7;
      w7x += d7 * nvx[b]; w7y += d7 * nvy[b];
      w8x += d8 * nvx[b]; w8y += d8 * nvy[b];
      w9x += d9 * nvx[b]; w9y += d9 * nvy[b];
    }
    const double wx[3] = {w7x, w8x, w9x}, wy[3] = {w7y, w8y, w9y};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double dw = dax * wx[q] + day * wy[q];
      acc[q * 9 + 0] += wx[q];
      acc[q * 9 + 1] += wy[q];
      acc[q * 9 + 2] += xi * wx[q];
      acc[q * 9 + 3] += eta * wx[q];
      acc[q * 9 + 4] += xi * wy[q];
      acc[q * 9 + 5] += eta * wy[q];
      acc[q * 9 + 6] += dw;
      acc[q * 9 + 7] += xi * dw;
      acc[q * 9 + 8] += eta * dw;
    }
    const double2 rk = kResidLds ? sres[n] : r[k];
    const double dr = dax * rk.x + day * rk.y;
    acc[KROW + 0] += dr;
    acc[KROW + 1] += xi * dr;
    acc[KROW + 2] += eta * dr;
  }
  {
    // 30 sums at once by halving exchanges: fewer lane moves than one
    // reduction per value, at every set edge
    double a32[32];
#pragma unroll
    for (int v = 0; v < 32; ++v) a32[v] = v < KROW + 3 ? acc[v] : 0.0;
    const double as = wave_sums<32>(a32);
    const int v = wave_sums_index<32>();
    if ((t & 1) == 0 && v < KROW + 3) sacc[t >> 6][v] = as;
  }
  __syncthreads();
  if (t < KROW + 3) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += sacc[w][t];
    if (t < KROW) A.krow[(size_t)tile * KROW + t] = s;
    else A.force[(size_t)tile * Q + 6 + (t - KROW)] = s;
  }
}

// Waves per SIMD the register allocation must allow.  The tile of a 32 x 32
// set with 512 threads and an overlap up to 2 is held to 128 registers, so
// that two tiles share a CU and one's barriers overlap the other's work: it
// spills a little (not in the sweep loop) but runs faster, 1.2-1.3x in
// float32 and 1.1-1.2x in float64.  Regions widened by more than 2 nodes
// keep one tile per CU.
template <typename T, int E, int NT, int OV>
constexpr int tile_waves_per_eu() { return E == 32 && NT == 512 && OV <= 2 ? 4 : 1; }

template <typename T, int E, int NT, int OV>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(tile_waves_per_eu<T, E, NT, OV>())))
void k_tile(Geo g, const float* __restrict__ ea,
                                             const uint8_t* __restrict__ mask, TileArgs A) {
  tile_body<T, E, NT, OV>(g, ea, mask, A, xcd_remap(blockIdx.x, gridDim.x));
}

// Fused launch over the tiles of several lattices with the same set edge and
// overlap: tile_lat maps a launch-wide tile index to its lattice entry.
template <typename T, int E, int NT, int OV>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(tile_waves_per_eu<T, E, NT, OV>())))
void k_tile_batch(const BatchEntry* __restrict__ B,
                                                   const int* __restrict__ tile_lat) {
  const int gt = xcd_remap(blockIdx.x, gridDim.x);
  const BatchEntry& e = B[tile_lat[gt]];
  tile_body<T, E, NT, OV>(e.g, e.ea, e.mask, e.ta, gt - e.tile0);
}

namespace {

__device__ __forceinline__ int lpk(int i, int j) { return i * (i + 1) / 2 + j; }

// Block-Jacobi preconditioner of one set: the symmetric pseudo-inverse of its
// 9x9 diagonal block, B^+ = S L^-T L^-1 S, from a Jacobi-scaled Cholesky
// factorisation S B S = L L^T that drops (zeroes) a mode whose pivot falls
// below 1e-9, i.e. a mode that is, to that level, a combination of the
// modes before it.
__device__ void block_pinv(const double* B, double* Binv) {
  double sc[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) sc[k] = B[k * Q + k] > 0.0 ? 1.0 / sqrt(B[k * Q + k]) : 0.0;
  double L[45];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double dkk = sc[k] * sc[k] * B[k * Q + k];
#pragma unroll
    for (int j = 0; j < k; ++j) dkk -= L[lpk(k, j)] * L[lpk(k, j)];
    const bool keep = sc[k] > 0.0 && dkk > 1e-9;
    const double lkk = keep ? sqrt(dkk) : 0.0;
    L[lpk(k, k)] = lkk;
#pragma unroll
    for (int i = k + 1; i < Q; ++i) {
      double v = sc[i] * sc[k] * B[i * Q + k];
#pragma unroll
      for (int j = 0; j < k; ++j) v -= L[lpk(i, j)] * L[lpk(k, j)];
      L[lpk(i, k)] = keep ? v / lkk : 0.0;
    }
  }
  // X = L^-1 (lower triangular; rows and columns of dropped modes stay 0)
  double X[45];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
#pragma unroll
    for (int i = j; i < Q; ++i) {
      const double lii = L[lpk(i, i)];
      double v = i == j ? 1.0 : 0.0;
#pragma unroll
      for (int k = j; k < i; ++k) v -= L[lpk(i, k)] * X[lpk(k, j)];
      X[lpk(i, j)] = lii > 0.0 ? v / lii : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < Q; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double v = 0.0;
#pragma unroll
      for (int k = i; k < Q; ++k) v += X[lpk(k, i)] * X[lpk(k, j)];
      v *= sc[i] * sc[j];
      Binv[i * Q + j] = v;
      Binv[j * Q + i] = v;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Upper-level blocks between neighbouring sets, from the rods their common
// boundary cuts: K[Im][Jl] = -sum_rods k (n . u_hat_m^I(a)) (n . u_hat_l^J(c)).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void offdiag_body(const Geo& g, const float* __restrict__ ea,
                                             const uint8_t* __restrict__ mask, const OffArgs& A,
                                             const int s) {
  using T2 = typename V2<T>::type;
  constexpr int MAXB = 2 * 64;
  __shared__ double G[MAXB][Q];
  __shared__ double H[MAXB][Q];
  if (A.ctrl->done) return;
  const T2* d = reinterpret_cast<const T2*>((A.ctrl->k & 1) ? A.d0 : A.d1);
  const int I = s % g.mx, J = s / g.mx;
  const int E = g.E;
  const int i0 = I * E, j0 = J * E, tw = min(E, g.nx - i0), th = min(E, g.ny - j0);
  const size_t plane = (size_t)(g.ny + 2) * g.pitch;
  const double inv_hs = 2.0 / E;
  const int t = threadIdx.x;

  for (int dir = 0; dir < 3; ++dir) {
    const int I2 = I + nb_di(dir), J2 = J + nb_dj(dir);
    if (I2 < 0 || I2 >= g.mx || J2 < 0 || J2 >= g.my) continue;
    const int oi0 = I2 * E, oj0 = J2 * E, otw = min(E, g.nx - oi0), oth = min(E, g.ny - oj0);
    const int nb = dir == 0 ? 2 * th - 1 : dir == 1 ? 2 * tw - 1 : 1;
    for (int b = t; b < nb; b += blockDim.x) {
      int ai, aj, ci, cj, plane_id;
      size_t kp;
      double nx_, ny_;
      if (dir == 0) {
        if (b < th) { ai = i0 + tw - 1; aj = j0 + b; ci = ai + 1; cj = aj; nx_ = 1.0; ny_ = 0.0; plane_id = 0; kp = pidx(g, ai, aj); }
        else { const int rr = b - th; ci = i0 + tw; cj = j0 + rr; ai = ci - 1; aj = cj + 1; nx_ = -0.5; ny_ = kS3; plane_id = 2; kp = pidx(g, ci, cj); }
      } else if (dir == 1) {
        if (b < tw) { ai = i0 + b; aj = j0 + th - 1; ci = ai; cj = aj + 1; nx_ = 0.5; ny_ = kS3; plane_id = 1; kp = pidx(g, ai, aj); }
        else { const int rr = b - tw + 1; ai = i0 + rr; aj = j0 + th - 1; ci = ai - 1; cj = aj + 1; nx_ = -0.5; ny_ = kS3; plane_id = 2; kp = pidx(g, ai, aj); }
      } else {
        ai = i0; aj = j0 + th - 1; ci = ai - 1; cj = aj + 1; nx_ = -0.5; ny_ = kS3; plane_id = 2; kp = pidx(g, ai, aj);
      }
      const double kr = (double)ea[plane_id * plane + kp];
      const size_t pa = pidx(g, ai, aj), pc = pidx(g, ci, cj);
      double xa, ya, xc, yc;
      set_coords(ai, aj, i0, j0, tw, th, inv_hs, xa, ya);
      set_coords(ci, cj, oi0, oj0, otw, oth, inv_hs, xc, yc);
      const bool fa = mask[pa] == 0, fc = mask[pc] == 0;
      const T2 da = d[pa], dc = d[pc];
      const double nda = nx_ * (double)da.x + ny_ * (double)da.y;
      const double ndc = nx_ * (double)dc.x + ny_ * (double)dc.y;
      const double ga[Q] = {nx_, ny_, xa * nx_, ya * nx_, xa * ny_, ya * ny_, nda, xa * nda, ya * nda};
      const double gc[Q] = {nx_, ny_, xc * nx_, yc * nx_, xc * ny_, yc * ny_, ndc, xc * ndc, yc * ndc};
#pragma unroll
      for (int m = 0; m < Q; ++m) {
        G[b][m] = fa ? kr * ga[m] : 0.0;
        H[b][m] = fc ? gc[m] : 0.0;
      }
    }
    __syncthreads();
    if (t < Q * Q) {
      const int m = t / Q, l = t % Q;
      double acc = 0.0;
      for (int b = 0; b < nb; ++b) acc -= G[b][m] * H[b][l];
      const int s2 = J2 * g.mx + I2;
      A.off[((size_t)s * NDIR + dir) * Q * Q + m * Q + l] = acc;
      A.off[((size_t)s2 * NDIR + dir + 3) * Q * Q + l * Q + m] = acc;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_offdiag(Geo g, const float* __restrict__ ea,
                                                 const uint8_t* __restrict__ mask, OffArgs A) {
  offdiag_body<T>(g, ea, mask, A, blockIdx.x);
}

// Fused launch over the sets of several lattices; set_lat maps a launch-wide
// set index to its lattice entry.
template <typename T>
__global__ __launch_bounds__(256) void k_offdiag_batch(const BatchEntry* __restrict__ B,
                                                       const int* __restrict__ set_lat) {
  const BatchEntry& e = B[set_lat[blockIdx.x]];
  offdiag_body<T>(e.g, e.ea, e.mask, e.oa, blockIdx.x - e.set0);
}

// ---------------------------------------------------------------------------
// Each set's diagonal upper-level block: the constant translation/gradient
// part plus the rows of the relaxation modes from the tile kernel (Eq. 6),
// and its pseudo-inverse for the block-Jacobi preconditioner.  One thread
// per set.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void blockinv_body(const Geo& g, const BlockArgs& A, const int s) {
  if (A.ctrl->done) return;
  if (s >= g.M) return;
  double B[Q * Q];
  const double* g1 = A.g1 + (size_t)s * 36;
  const double* kr = A.krow + (size_t)s * KROW;
  for (int m = 0; m < 6; ++m)
    for (int l = 0; l < 6; ++l) B[m * Q + l] = g1[m * 6 + l];
  for (int q = 0; q < 3; ++q)
    for (int l = 0; l < 6; ++l) { B[(6 + q) * Q + l] = kr[q * 9 + l]; B[l * Q + 6 + q] = kr[q * 9 + l]; }
  for (int q = 0; q < 3; ++q)
    for (int p = 0; p < 3; ++p) B[(6 + q) * Q + 6 + p] = 0.5 * (kr[q * 9 + 6 + p] + kr[p * 9 + 6 + q]);
  double* bd = A.bdiag + (size_t)s * Q * Q;
  for (int v = 0; v < Q * Q; ++v) bd[v] = B[v];
  double Bi[Q * Q];
  block_pinv(B, Bi);
  double* bi = A.binv + (size_t)s * Q * Q;
  for (int v = 0; v < Q * Q; ++v) bi[v] = Bi[v];
}

// BLOCKINV_SETS sets per wave (the rest of its lanes idle): the per-set work
// is one long dependent chain per lane, and its strided loads and stores of
// whole 9 x 9 blocks touch one cache line per lane, so fewer sets per wave,
// on more CUs, finish a little sooner.
constexpr int BLOCKINV_SETS = 16;
__global__ __launch_bounds__(64) void k_blockinv(Geo g, BlockArgs A) {
  if (threadIdx.x >= BLOCKINV_SETS) return;
  blockinv_body(g, A, blockIdx.x * BLOCKINV_SETS + threadIdx.x);
}

__global__ __launch_bounds__(64) void k_blockinv_batch(const BatchEntry* __restrict__ B,
                                                       const int* __restrict__ set_lat,
                                                       int nsets) {
  if (threadIdx.x >= BLOCKINV_SETS) return;
  const int gs = blockIdx.x * BLOCKINV_SETS + threadIdx.x;
  if (gs >= nsets) return;
  const BatchEntry& e = B[set_lat[gs]];
  blockinv_body(e.g, e.ba, gs - e.set0);
}

// ---------------------------------------------------------------------------
// Upper level: stop test of Eq. 19 and block-Jacobi PCG on Eq. 8.
//
// The grid is co-resident (at most one workgroup per CU).  Workgroup w owns
// the sets [s0, s1) and keeps their PCG vectors in LDS.  Only two things
// cross workgroups inside the kernel: the published z and p of each set
// (read by the neighbouring sets' products) and the reduction partials.
// Those are written and read with agent-scope relaxed atomics, which go to
// the device-coherent level, and every wave waits for its stores to
// complete before the barrier arrival; no L2-wide fence is needed.
// ---------------------------------------------------------------------------
namespace {

__device__ __forceinline__ void pub_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double pub_load(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide sum of up to REDW values, which is also the grid barrier.
// Workgroup w publishes its partials in slot `slot`, waits for all of its
// stores (the partials and any values published before the call), then
// arrives on a two-level counter (eight group counters, then a root); every
// workgroup waits until the root shows all arrivals of generation `gen` and
// then adds the partials in workgroup order, so all threads of all
// workgroups get the same bits.  A workgroup can run at most one sum ahead of
// the slowest, hence two slots.  Bounded: after spin_limit polls the error
// flag is raised and every later call returns false at once, so the grid
// always drains.  With one workgroup the partials are left in sv and no
// memory round trip is made.
template <int NV>
__device__ bool grid_publish_wait(const double (&v)[NV], double* red, unsigned* flags,
                                  unsigned gen, int slot, Ctrl* c, int wid, int nwg,
                                  unsigned spin, double* sslot, double* sv) {
  __shared__ int ok;
  __shared__ double wsum[NV][COARSE_NT / 64];
  static_assert(NV <= REDW, "too many values for one grid sum");
  // the workgroup's sums of the NV values: one barrier for all of them
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double ws = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) wsum[k][threadIdx.x >> 6] = ws;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double bs = 0.0;
#pragma unroll
    for (int w = 0; w < COARSE_NT / 64; ++w) bs += wsum[threadIdx.x][w];
    if (nwg == 1) sv[threadIdx.x] = bs;
    else pub_store(&red[((size_t)slot * REDW + threadIdx.x) * COARSE_MAX_WG + wid], bs);
  }
  if (nwg == 1) {
    __syncthreads();
    return true;
  }
  // one wait covers every store of this workgroup: published values and partials
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    // Arrival: one atomic add on the counter of the workgroup's group (the
    // workgroups w with the same w mod 8); the group's last arrival adds one
    // to the root counter, which every workgroup polls.  The counters only
    // grow from zero (they are cleared with the solve's state), so after
    // grid sum number gen the root holds gen times the number of groups.
    const int grp = wid % BAR_GROUPS;
    const int gsize = nwg / BAR_GROUPS + (grp < nwg % BAR_GROUPS ? 1 : 0);
    const unsigned ngrp = (unsigned)min(nwg, BAR_GROUPS);
    unsigned* root = flags + BAR_GROUPS * 16;
    const unsigned old = __hip_atomic_fetch_add(flags + grp * 16, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if ((old + 1u) % (unsigned)gsize == 0u)
      __hip_atomic_fetch_add(root, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = gen * ngrp;
    int good = 1;
    unsigned n = 0;
    for (;;) {
      // the root and the error flag are loaded together: one round trip a poll
      const unsigned rv = __hip_atomic_load(root, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int err = __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const bool done = (int)(rv - target) >= 0;
      if (err != 0 || (!done && ++n > spin)) {
        __hip_atomic_store(&c->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      if (done) break;
      __builtin_amdgcn_s_sleep(1);
    }
    ok = good;
  }
  __syncthreads();
  (void)sslot;
  return ok != 0;
}

// After a grid sum: add the published partials into sv, copy the
// neighbours' published window values into LDS, and (agg_nvec > 0) gather
// the coarse-space restrictions: for each of agg_nvec vectors, entry
// (aggregate a, mode k) is the sum, in workgroup order, of partial
// agg_k0 + 6 v + k of the agg_g workgroups of aggregate a.  The partials are
// stored value-major ([slot][value][workgroup]) so that these loads are
// contiguous across lanes.  Thread t takes workgroup t's partials; the four
// waves' sums are added in wave order, the same tree in every workgroup, so
// every workgroup gets the same bits.  All loads are issued before any is
// used, so they take one memory round trip together.  Only the collecting
// threads write sv / s_c; the caller synchronises.
template <int NV, int NVEC = 1, int WB = 4>
__device__ void grid_collect_window(const double* red, int slot, int nwg, double* sv,
                                    double* dst, const double* src, int n,
                                    int agg_k0 = 0, int agg_nvec = 0, int agg_g = 1,
                                    int naggr = 0, double* s_c = nullptr) {
  constexpr int NWV = COARSE_NT / 64;
  constexpr int CB = (NVEC * 6 * AGG_MAX + COARSE_NT - 1) / COARSE_NT;
  static_assert(COARSE_NT == COARSE_MAX_WG, "one collecting thread per workgroup");
  __shared__ double wpart[NV][NWV];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (nwg <= 1) return;
  const double* rs = red + (size_t)slot * REDW * COARSE_MAX_WG;
  // Every load is issued unconditionally, with its index clamped into the
  // buffer, and what a lane does not need is dropped by a select later.  A
  // load under a branch lets the compiler pull its first use next to it,
  // which costs one memory round trip per load; this way all of them are in
  // flight together.
  double pv[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) pv[k] = pub_load(&rs[(size_t)k * COARSE_MAX_WG + t]);
  // coarse-space restrictions: entry e = (6 v + k) naggr + a, for e = t, t + NT
  double cv[CB][AGG_GMAX];
  const int ctot = agg_nvec * 6 * naggr;
  const int na = max(naggr, 1);
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    const int e = t + b * COARSE_NT < ctot ? t + b * COARSE_NT : 0;
    const int vk = e / na, ag = e - vk * na;
    const double* col = rs + (size_t)(agg_k0 + vk) * COARSE_MAX_WG;
#pragma unroll
    for (int j = 0; j < AGG_GMAX; ++j) cv[b][j] = pub_load(&col[min(ag * agg_g + j, COARSE_MAX_WG - 1)]);
  }
  // the window: its first WB * NT entries (normally all of it) are loaded
  // here, outside any loop, so that they share the round trip above
  const bool win_on = src != nullptr && n > 0;
  double wv_[WB];
  if (win_on) {
#pragma unroll
    for (int b = 0; b < WB; ++b) wv_[b] = pub_load(&src[min(t + b * COARSE_NT, n - 1)]);
  }
  if (win_on) {
#pragma unroll
    for (int b = 0; b < WB; ++b)
      if (t + b * COARSE_NT < n) dst[t + b * COARSE_NT] = wv_[b];
    for (int base = WB * COARSE_NT; base < n; base += WB * COARSE_NT) {
#pragma unroll
      for (int b = 0; b < WB; ++b) wv_[b] = pub_load(&src[min(base + t + b * COARSE_NT, n - 1)]);
#pragma unroll
      for (int b = 0; b < WB; ++b) {
        const int e = base + t + b * COARSE_NT;
        if (e < n) dst[e] = wv_[b];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double x = wave_sum(t < nwg ? pv[k] : 0.0);
    if (lane == 0) wpart[k][wv] = x;
  }
  if (ctot > 0) {
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int e = t + b * COARSE_NT;
      const int vk = e / na, ag = e - vk * na;
      double sum = 0.0;
#pragma unroll
      for (int j = 0; j < AGG_GMAX; ++j) sum += j < agg_g && ag * agg_g + j < nwg ? cv[b][j] : 0.0;
      if (e < ctot) s_c[(vk / 6) * 6 * AGG_MAX + 6 * ag + vk % 6] = sum;
    }
  }
  __syncthreads();
  if (t < NV) {
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < NWV; ++q) sum += wpart[t][q];
    sv[t] = sum;
  }
}


// Coarse space of the upper-level preconditioner.  Aggregates are runs of
// agg_sets consecutive sets (whole workgroups); each carries six affine
// displacement fields about its centroid (X, Y), scaled by 1/E, written in
// the set modes 1-6: for set s with tile centroid (x_s, y_s) and
// dx = (x_s - X)/E, dy = (y_s - Y)/E the field u_x = (x - X)/E is
// 0.5 * mode 3 + dx * mode 1, and likewise for the other three gradients.
// The preconditioner is then the additive two-level B^+ + P0 A0^+ P0^T with
// A0 = P0^T K_a P0, which involves only the constant modes 1-6.
__device__ __forceinline__ void agg_coef(const Geo& g, const double* agg_xy, int agg_sets, int s,
                                         double& dx, double& dy) {
  const int a = s / agg_sets;
  const int I = s % g.mx, J = s / g.mx;
  const int i0 = I * g.E, j0 = J * g.E;
  const int tw = min(g.E, g.nx - i0), th = min(g.E, g.ny - j0);
  const double ic = i0 + 0.5 * (tw - 1), jc = j0 + 0.5 * (th - 1);
  dx = (ic + 0.5 * jc - agg_xy[2 * a]) / g.E;
  dy = (jc * kS3 - agg_xy[2 * a + 1]) / g.E;
}

// P0^T: the contribution of row (set, mode l) holding v to the six
// aggregate-mode entries c[0..5].
__device__ __forceinline__ void agg_restrict(int l, double v, double dx, double dy, double (&c)[6]) {
  if (l == 0) { c[0] += v; c[2] += dx * v; c[3] += dy * v; }
  else if (l == 1) { c[1] += v; c[4] += dx * v; c[5] += dy * v; }
  else if (l < 6) c[l] += 0.5 * v;
}

// P0: the value on row (set, mode l) of the aggregate-mode vector y[0..5].
__device__ __forceinline__ double agg_prolong(int l, const double* y, double dx, double dy) {
  if (l == 0) return y[0] + dx * y[2] + dy * y[3];
  if (l == 1) return y[1] + dx * y[4] + dy * y[5];
  if (l < 6) return 0.5 * y[l];
  return 0.0;
}

// y[v][r] = (A0^+ c[v]) on the rows r = 6 (a - a_lo) + k of the aggregates
// a_lo .. a_lo + nwa - 1.  Their rows of A0^+ are in LDS column by column
// (entry (r, j) at rows[j * 6 nwa + r]).  Each lane takes a row and a run of
// columns: with at most 16 (32) rows in any window of the lattice (nr_max)
// a wave holds four (two) runs side by side, and the four waves take
// further runs, so no lane waits on a cross-lane sum.  The runs meet in
// `part` ([runs][2][rows per pass]) and are added in run order; the runs
// depend only on the lattice, so every workgroup gets the same bits for a
// shared aggregate.  Ends synchronised.
constexpr int SOLVE_STEP = 6;
__device__ void agg_window_solve(const double* rows, int naggr, int nwa, int nr_max,
                                 const double* c, double* y, int nvec, double* part) {
  constexpr int NWV = COARSE_NT / 64;
  const int n = 6 * naggr, nr = 6 * nwa;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int PH = nr_max <= 16 ? 4 : nr_max <= 32 ? 2 : 1;
  const int RP = 64 / PH;                   // rows per pass
  const int ph = lane / RP, rl = lane - RP * ph;
  const int nq = NWV * PH, q = wv * PH + ph;
  const int cq = (n + nq - 1) / nq;
  const int jb = min(n, q * cq), je = min(n, jb + cq);
  for (int rb = 0; rb < nr; rb += RP) {
    const int r = min(rb + rl, nr - 1);
    for (int v = 0; v < nvec; ++v) {
      const double* cv = c + v * 6 * AGG_MAX;
      // SOLVE_STEP columns per step, all loads issued before any product
      // (the step is bound by LDS latency); past je the column index is
      // clamped and the factor is zero
      double acc[2] = {0.0, 0.0};
      for (int j0 = jb; j0 < je; j0 += SOLVE_STEP) {
        double rv[SOLVE_STEP], cc[SOLVE_STEP];
#pragma unroll
        for (int k = 0; k < SOLVE_STEP; ++k) {
          const int j = min(j0 + k, je - 1);
          rv[k] = rows[(size_t)j * nr + r];
          const double cj = cv[j];
          cc[k] = j0 + k < je ? cj : 0.0;
        }
#pragma unroll
        for (int k = 0; k < SOLVE_STEP; ++k) acc[k & 1] += rv[k] * cc[k];
      }
      part[(q * 2 + v) * RP + rl] = acc[0] + acc[1];
    }
    __syncthreads();
    if ((int)threadIdx.x < RP * nvec) {
      const int v = threadIdx.x / RP, l = threadIdx.x - RP * v;
      if (rb + l < nr) {
        // the runs' partials, four loads in flight at a time
        double sum = 0.0;
        for (int q0 = 0; q0 < nq; q0 += 4) {
          double pr[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) pr[k] = part[(min(q0 + k, nq - 1) * 2 + v) * RP + l];
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (q0 + k < nq) sum += pr[k];
        }
        y[v * 6 * AGG_MAX + rb + l] = sum;
      }
    }
    __syncthreads();
  }
}

// (K_a v) for one row of the workgroup's own sets, v from the LDS window that
// starts at set w0.  bd / ob point at the own sets' diagonal and neighbour
// blocks (an LDS copy or global memory), indexed from set s0.
template <bool kWide>
__device__ __forceinline__ double coarse_row(const Geo& g, const double* bd, const double* ob,
                                             int s, int s0, int m, const double* lv, int w0) {
  const int I = s % g.mx, J = s / g.mx;
  const double* b = bd + (size_t)(s - s0) * Q * Q + m * Q;
  const double* pv = lv + (size_t)(s - w0) * Q;
  double q = 0.0;
#pragma unroll
  for (int l = 0; l < Q; ++l) q += b[l] * pv[l];
  // kWide: branch-free over the six neighbours (an absent one reads the
  // set's own window entries and contributes exact zeros), so that all 63
  // block loads can be in flight at once when the blocks are in global
  // memory.  It needs about 126 more registers; the batched kernel, held to
  // 256, skips absent neighbours instead.
#pragma unroll
  for (int dir = 0; dir < NDIR; ++dir) {
    const int I2 = I + nb_di(dir), J2 = J + nb_dj(dir);
    const bool ok = I2 >= 0 && I2 < g.mx && J2 >= 0 && J2 < g.my;
    if (!kWide && !ok) continue;
    const double* o = ob + ((size_t)(s - s0) * NDIR + dir) * Q * Q + m * Q;
    const double* pn = lv + (size_t)((ok ? J2 * g.mx + I2 : s) - w0) * Q;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const double ov = o[l];
      q += (ok ? ov : 0.0) * pn[l];
    }
  }
  return q;
}

// One row of B^+ v for the own set s, v (own rows) in LDS at lv (set s0 first).
__device__ __forceinline__ double pinv_row(const double* bi, int s, int s0, int m,
                                           const double* lv) {
  const double* b = bi + (size_t)(s - s0) * Q * Q + m * Q;
  const double* v = lv + (size_t)(s - s0) * Q;
  double z = 0.0;
#pragma unroll
  for (int l = 0; l < Q; ++l) z += b[l] * v[l];
  return z;
}

}  // namespace

// m += P0 A0^+ P0^T w on the window: solve the window aggregates' rows of
// A0^+ against the gathered restriction s_c, then add the prolongation to
// the window copy of m (modes 1-6).  Ends synchronised.
__device__ void coarse_space_correction(const CoarseArgs& A, int nwa, int win,
                                        const double* s_c, double* s_y, double* lw,
                                        const double* lrows, const double* ldxy,
                                        double* lpart, int nr_max) {
  agg_window_solve(lrows, A.naggr, nwa, nr_max, s_c, s_y, 1, lpart);
  // one thread per window set: its aggregate's six values, then modes 1-6
  for (int sl = threadIdx.x; sl < win; sl += COARSE_NT) {
    const double* d = ldxy + 3 * sl;
    const double dx = d[0], dy = d[1];
    const double* y = s_y + 6 * (int)d[2];
    double* m = lw + (size_t)sl * Q;
#pragma unroll
    for (int l = 0; l < 6; ++l) m[l] += agg_prolong(l, y, dx, dy);
  }
  __syncthreads();
}

// Dynamic LDS of the upper-level kernel: a window of the set vectors, the
// own rows of the vector being preconditioned and the window aggregates'
// rows of the coarse-space inverse, plus (when they fit) the own sets' PCG
// vectors and their blocks.
size_t coarse_lds_bytes(const Geo& g, int nwg, int vec_lds, int blk_lds, int two_level) {
  const size_t spw = (size_t)(g.M + nwg - 1) / nwg;
  const size_t win = std::min((size_t)g.M, spw + 2 * (size_t)g.mx + 2);
  size_t b = (spw + win) * Q * sizeof(double);
  if (two_level) {
    const AggLayout al = agg_layout(g.M, g.mx, nwg);
    b += (size_t)6 * al.nwa_max * 6 * al.naggr * sizeof(double);   // coarse-space rows
    b += 3 * win * sizeof(double);                                  // P0 entries of the window
    b += AGG_PART * sizeof(double);                                 // partial sums of its solve
  }
  if (vec_lds) b += 8 * spw * Q * sizeof(double);
  if (blk_lds) b += spw * (NDIR + 2) * Q * Q * sizeof(double);
  return b;
}

// A plain load that the compiler keeps where it is written: a relaxed
// atomic load at workgroup scope is an ordinary cached load, but it is not
// moved next to its first use, so a batch of them shares one round trip.
__device__ __forceinline__ double stage_load(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// n doubles from global memory into LDS, LDS_COPY_BATCH loads in flight per
// thread (a copy loop with one load per step waits a full memory round trip
// per step).
constexpr int LDS_COPY_BATCH = 16;
__device__ __forceinline__ void copy_to_lds(double* dst, const double* src, int n) {
  const int t = threadIdx.x;
  for (int base = 0; base < n; base += LDS_COPY_BATCH * COARSE_NT) {
    double v[LDS_COPY_BATCH];
#pragma unroll
    for (int b = 0; b < LDS_COPY_BATCH; ++b) v[b] = stage_load(&src[min(base + t + b * COARSE_NT, n - 1)]);
#pragma unroll
    for (int b = 0; b < LDS_COPY_BATCH; ++b)
      if (base + t + b * COARSE_NT < n) dst[base + t + b * COARSE_NT] = v[b];
  }
}

// An r x n row-major block from global memory into LDS column by column
// (element (i, j) to dst[j * r + i]), LDS_COPY_BATCH loads in flight per
// thread.
__device__ __forceinline__ void copy_to_lds_transposed(double* dst, const double* src, int r, int n) {
  const int t = threadIdx.x, tot = r * n;
  for (int base = 0; base < tot; base += LDS_COPY_BATCH * COARSE_NT) {
    double v[LDS_COPY_BATCH];
#pragma unroll
    for (int b = 0; b < LDS_COPY_BATCH; ++b) v[b] = stage_load(&src[min(base + t + b * COARSE_NT, tot - 1)]);
#pragma unroll
    for (int b = 0; b < LDS_COPY_BATCH; ++b) {
      const int e = base + t + b * COARSE_NT;
      if (e < tot) dst[(size_t)(e % n) * r + e / n] = v[b];
    }
  }
}

// Upper-level kernel.  Pipelined block-Jacobi PCG (the Ghysels-Vanroose
// recurrences): per iteration one grid sum carries both dot products and
// orders the publication of m = B^+ w, whose neighbour values the product
// n = K_a m needs, so one grid synchronisation per iteration.
template <bool kWide>
__device__ __forceinline__ void coarse_body(const Geo& g, const CoarseArgs& A, const int w,
                                            const int nwg) {
  extern __shared__ double lds[];
  __shared__ double sslot[COARSE_NT / 64];
  __shared__ double sv[REDW];
  Ctrl* ctrl = A.ctrl;
  // the control words are read together (one round trip), then tested
  const int done = __hip_atomic_load(&ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const unsigned base = __hip_atomic_load(&ctrl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const int iter = __hip_atomic_load(&ctrl->k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (done) return;
  const int t = threadIdx.x;
  const int M = g.M;
  const int spw = (M + nwg - 1) / nwg;
  const int s0 = min(M, w * spw), s1 = min(M, s0 + spw), ns = s1 - s0;
  const int w0 = max(0, s0 - g.mx - 1), w1 = min(M, s1 + g.mx + 1);
  const int win = ns > 0 ? w1 - w0 : 0;
  const int nrow = ns * Q;
  const unsigned spin = A.spin_limit;
  // coarse space: restrictions (two vectors at the start) and the window
  // aggregates' corrections
  const bool two = A.naggr > 0;
  __shared__ double s_c[2 * 6 * AGG_MAX];
  __shared__ double s_y[2 * 6 * AGG_MAX];
  const int a_lo = two && win > 0 ? w0 / A.agg_sets : 0;
  const int nwa = two && win > 0 ? (w1 - 1) / A.agg_sets - a_lo + 1 : 0;
  unsigned nsync = 0;
  int slot = 0;
  const int wmax = min(M, spw + 2 * g.mx + 2);
  double* lown = lds;                          // own rows of the vector being preconditioned
  double* lw1 = lown + (size_t)spw * Q;        // window (first vector)
  // The start's second window (u0) reuses the first: the first holds the
  // previous coefficients only until the start's grid sum.
  double* lw2 = lw1;
  double* lrows = lw1 + (size_t)wmax * Q;     // window aggregates' rows of A0^+
  const AggLayout alay = agg_layout(M, g.mx, nwg);
  const size_t nrows_lds = two ? (size_t)6 * alay.nwa_max * 6 * alay.naggr : 0;
  double* ldxy = lrows + nrows_lds;                     // [wmax][3]: dx, dy, aggregate
  double* lpart = ldxy + (two ? (size_t)3 * wmax : 0);  // [4][2][64] partial sums of the solve
  double* lnext = lpart + (two ? (size_t)AGG_PART : 0);
  const size_t r0 = (size_t)s0 * Q;            // first own row
  // Own-row vectors, touched only by the owning thread: in LDS when they fit,
  // else in global memory.  All are indexed from the workgroup's first row.
  double *vx, *vr, *vu, *vw, *vz, *vq, *vs, *vp;
  double* vn = A.cn + r0;
  if (A.vec_lds) {
    double* b = lnext;
    vx = b; vr = b + (size_t)spw * Q; vu = b + 2 * (size_t)spw * Q; vw = b + 3 * (size_t)spw * Q;
    vz = b + 4 * (size_t)spw * Q; vq = b + 5 * (size_t)spw * Q; vs = b + 6 * (size_t)spw * Q;
    vp = b + 7 * (size_t)spw * Q;
    lnext += 8 * (size_t)spw * Q;
  } else {
    vx = A.a + r0; vr = A.cr + r0; vu = A.cu + r0; vw = A.cw + r0; vz = A.cz + r0;
    vq = A.cq + r0; vs = A.cs + r0; vp = A.cp + r0;
  }
  // own sets' blocks (diagonal, six neighbours, pseudo-inverse)
  const double* bd = A.bdiag + (size_t)s0 * Q * Q;
  const double* ob = A.off + (size_t)s0 * NDIR * Q * Q;
  const double* bi = A.binv + (size_t)s0 * Q * Q;
  // Staged into LDS once per launch: the own sets' blocks (when they fit)
  // and the window aggregates' rows of A0^+ (column by column).
  if (A.blk_lds) {
    double* lb = lnext;
    copy_to_lds(lb, bd, ns * Q * Q);
    copy_to_lds(lb + (size_t)spw * Q * Q, bi, ns * Q * Q);
    copy_to_lds(lb + 2 * (size_t)spw * Q * Q, ob, ns * NDIR * Q * Q);
    bd = lb;
    bi = lb + (size_t)spw * Q * Q;
    ob = lb + 2 * (size_t)spw * Q * Q;
  }
  if (two)
    copy_to_lds_transposed(lrows, A.agg_inv + (size_t)36 * a_lo * A.naggr, 6 * nwa, 6 * A.naggr);
  __syncthreads();
  if (two) {   // P0's entries of the window, once per launch
    for (int e = t; e < win; e += COARSE_NT) {
      double dx, dy;
      agg_coef(g, A.agg_xy, A.agg_sets, w0 + e, dx, dy);
      ldxy[3 * e] = dx;
      ldxy[3 * e + 1] = dy;
      ldxy[3 * e + 2] = (double)((w0 + e) / A.agg_sets - a_lo);
    }
    __syncthreads();
  }

  // --- start.  The warm start x0 = theta a_prev takes the previous solve's
  //     coefficients scaled by the step that minimises the upper-level
  //     energy along them (so the outer energy still decreases).  With
  //     y = K_a a_prev:  r0 = P - theta y,  u0 = B^+ P - theta B^+ y, and
  //     theta = (a_prev . P) / (a_prev . y).  One grid sum carries theta's
  //     two dot products, the stop test's four norm sums, and orders the
  //     publication of B^+ P and B^+ y.
  const bool warm = A.warm && iter > 0;
  if (warm) copy_to_lds(lw1, A.a + (size_t)w0 * Q, win * Q);
  else
    for (int e = t; e < win * Q; e += COARSE_NT) lw1[e] = 0.0;
  __syncthreads();
  // [0..3] stop-test norms, [4..5] theta's dot products, [6] P . B^+ P,
  // [7..12] P0^T P, [13..18] P0^T y (coarse space)
  double red6[19];
#pragma unroll
  for (int v = 0; v < 19; ++v) red6[v] = 0.0;
  double cP[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, cY[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int s = s0 + t; s < s1; s += COARSE_NT) {
#pragma unroll
    for (int v = 0; v < NRM; ++v) red6[v] += A.nrm[(size_t)s * NRM + v];
  }
  for (int e = t; e < nrow; e += COARSE_NT) {
    const int s = s0 + e / Q, m = e % Q;
    const double y = warm ? coarse_row<kWide>(g, bd, ob, s, s0, m, lw1, w0) : 0.0;
    const double aprev = lw1[(size_t)(s0 - w0) * Q + e];
    red6[4] += aprev * A.force[r0 + e];
    red6[5] += aprev * y;
    vn[e] = y;                   // keep y for r0
    lown[e] = A.force[r0 + e];
    if (two && m < 6) {
      double dx, dy;
      agg_coef(g, A.agg_xy, A.agg_sets, s, dx, dy);
      agg_restrict(m, A.force[r0 + e], dx, dy, cP);
      agg_restrict(m, y, dx, dy, cY);
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    red6[7 + k] = cP[k];
    red6[13 + k] = cY[k];
  }
  __syncthreads();
  for (int e = t; e < nrow; e += COARSE_NT) {
    const int s = s0 + e / Q, m = e % Q;
    const double v = pinv_row(bi, s, s0, m, lown);
    pub_store(&A.pub0[r0 + e], v);    // B^+ P
    vz[e] = v;
    red6[6] += lown[e] * v;           // P . B^+ P: the zero-start PCG residual
  }
  __syncthreads();
  for (int e = t; e < nrow; e += COARSE_NT) lown[e] = vn[e];
  __syncthreads();
  for (int e = t; e < nrow; e += COARSE_NT) {
    const int s = s0 + e / Q, m = e % Q;
    const double v = pinv_row(bi, s, s0, m, lown);
    pub_store(&A.pub1[r0 + e], v);    // B^+ y
    vq[e] = v;
  }
  if (!grid_publish_wait<19>(red6, A.red, A.flags, base + (++nsync), slot, ctrl, w, nwg, spin, sslot, sv))
    return;
  grid_collect_window<7, 2>(A.red, slot, nwg, sv, nullptr, nullptr, 0, 7, two ? 2 : 0, A.agg_g,
                            A.naggr, s_c);
  if (two && nwg == 1 && t < 12) s_c[(t / 6) * 6 * AGG_MAX + t % 6] = sv[7 + t];
  slot ^= 1;
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 7; ++v) red6[v] = sv[v];
  const double gamma_zero = red6[6];
  {
    const double R1 = red6[2] > 0.0 ? red6[0] / red6[2] : red6[0];
    const double R2 = red6[3] > 0.0 ? sqrt(red6[1] / red6[3]) : sqrt(red6[1]);
    const double R = fmax(R1, R2);
    int status = -100;   // continue
    if (!isfinite(red6[0]) || !isfinite(red6[1]) || !isfinite(red6[2]) || !isfinite(red6[3])) status = -6;
    else if (R <= A.rtol) status = 0;
    else if (iter >= A.max_iters) status = -3;
    if (w == 0 && t == 0) {
      if (A.hist) A.hist[iter] = R;
      ctrl->r1 = R1;
      ctrl->r2 = R2;
      if (status != -100) {
        ctrl->status = status;
        ctrl->iters = iter;
        ctrl->done = 1;
        ctrl->bar_gen = base + nsync;
      }
    }
    if (status != -100) return;
  }
  const double theta = (warm && red6[5] > 0.0 && red6[4] > 0.0) ? red6[4] / red6[5] : 0.0;
  // coarse-space parts of B^+ P and B^+ y on the window's aggregates
  if (two) {
    agg_window_solve(lrows, A.naggr, nwa, 6 * alay.nwa_max, s_c, s_y, 2, lpart);
  }
  // x0, r0, u0 (own) and u0 over the window, then w0 = K_a u0
  // (the published values are loaded four rows per thread at a time, so
  // that their round trips overlap)
  for (int base = 0; base < win * Q; base += 4 * COARSE_NT) {
    double p0[4], p1[4];
    const double* g0 = A.pub0 + (size_t)w0 * Q;
    const double* g1 = A.pub1 + (size_t)w0 * Q;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int e = min(base + t + c * COARSE_NT, win * Q - 1);
      p0[c] = pub_load(&g0[e]);
      p1[c] = pub_load(&g1[e]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int e = base + t + c * COARSE_NT;
      if (e >= win * Q) continue;
      double v = p0[c] - theta * p1[c];
      if (two && e % Q < 6) {
        const double* d = ldxy + 3 * (e / Q);
        const int al = (int)d[2];
        double yv[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) yv[k] = s_y[6 * al + k] - theta * s_y[6 * AGG_MAX + 6 * al + k];
        v += agg_prolong(e % Q, yv, d[0], d[1]);
      }
      lw2[e] = v;
    }
  }
  __syncthreads();
  for (int e = t; e < nrow; e += COARSE_NT) {
    vx[e] = warm ? theta * A.a[r0 + e] : 0.0;
    vr[e] = A.force[r0 + e] - theta * vn[e];
    vu[e] = lw2[(size_t)(s0 - w0) * Q + e];     // M^-1 r0 on the own rows
  }
  __syncthreads();
  for (int e = t; e < nrow; e += COARSE_NT) {
    const double wv = coarse_row<kWide>(g, bd, ob, s0 + e / Q, s0, e % Q, lw2, w0);
    vw[e] = wv;
    vz[e] = 0.0;
    vq[e] = 0.0;
    vs[e] = 0.0;
    vp[e] = 0.0;
  }
  __syncthreads();

  // --- pipelined PCG iterations
  double gamma0 = 0.0, gamma_prev = 0.0, alpha_prev = 0.0;
  int it = 0;
  if (nrow <= COARSE_NT) {
    // One row per thread: the row's blocks, pseudo-inverse row and PCG
    // vectors live in registers; only the neighbour window is read from LDS.
    const bool own = t < nrow;
    const int s = s0 + (own ? t / Q : 0), m = t % Q;
    const int I = s % g.mx, J = s / g.mx;
    double brow[Q], birow[Q], orow[NDIR][Q];
    int noff[NDIR];
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      brow[l] = own ? bd[(size_t)(s - s0) * Q * Q + m * Q + l] : 0.0;
      birow[l] = own ? bi[(size_t)(s - s0) * Q * Q + m * Q + l] : 0.0;
    }
#pragma unroll
    for (int dir = 0; dir < NDIR; ++dir) {
      const int I2 = I + nb_di(dir), J2 = J + nb_dj(dir);
      const bool ok = own && I2 >= 0 && I2 < g.mx && J2 >= 0 && J2 < g.my;
      noff[dir] = ok ? (J2 * g.mx + I2 - w0) * Q : (s - w0) * Q;
#pragma unroll
      for (int l = 0; l < Q; ++l)
        orow[dir][l] = ok ? ob[((size_t)(s - s0) * NDIR + dir) * Q * Q + m * Q + l] : 0.0;
    }
    const int sown = (s - w0) * Q, sset = (s - s0) * Q;
    double x = own ? vx[t] : 0.0, r = own ? vr[t] : 0.0, u = own ? vu[t] : 0.0;
    double wv = own ? vw[t] : 0.0, z = 0.0, q = 0.0, sv_ = 0.0, p = 0.0;
    double rdx = 0.0, rdy = 0.0;
    if (two && own) agg_coef(g, A.agg_xy, A.agg_sets, s, rdx, rdy);
    for (;; ++it) {
      // the two dot products and the coarse-space restriction of w
      double gd[8] = {r * u, wv * u, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (two && own) {
        double c6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        agg_restrict(m, wv, rdx, rdy, c6);
#pragma unroll
        for (int k = 0; k < 6; ++k) gd[2 + k] = c6[k];
      }
      if (own) lown[t] = wv;
      __syncthreads();
      double mv = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) mv += birow[l] * lown[sset + l];
      double* mpub = (it & 1) ? A.pub0 : A.pub2;
      if (own) {
        if (nwg == 1) lw1[t] = mv;
        else pub_store(&mpub[r0 + t], mv);
      }
      if (!grid_publish_wait<8>(gd, A.red, A.flags, base + (++nsync), slot, ctrl, w, nwg, spin, sslot, sv))
        return;
      grid_collect_window<2, 1, 4>(A.red, slot, nwg, sv, lw1, mpub + (size_t)w0 * Q, win * Q, 2,
                             two ? 1 : 0, A.agg_g, A.naggr, s_c);
      if (two && nwg == 1 && t < 6) s_c[t] = sv[2 + t];
      slot ^= 1;
      __syncthreads();
      const double gamma = sv[0], delta = sv[1];
      if (it == 0) gamma0 = A.coarse_ref ? gamma_zero : gamma;
      if (it >= A.coarse_iters || !(gamma > 0.0) ||
          !(gamma > A.coarse_rtol * A.coarse_rtol * gamma0)) break;
      double alpha, beta;
      if (it == 0) {
        beta = 0.0;
        alpha = delta > 0.0 ? gamma / delta : 0.0;
      } else {
        beta = gamma / gamma_prev;
        const double den = delta - beta * gamma / alpha_prev;
        alpha = den > 0.0 ? gamma / den : 0.0;
      }
      if (!(alpha > 0.0)) break;
      if (two) coarse_space_correction(A, nwa, win, s_c, s_y, lw1, lrows, ldxy, lpart, 6 * alay.nwa_max);
      double n = 0.0;
#pragma unroll
      for (int l = 0; l < Q; ++l) n += brow[l] * lw1[sown + l];
#pragma unroll
      for (int dir = 0; dir < NDIR; ++dir)
#pragma unroll
        for (int l = 0; l < Q; ++l) n += orow[dir][l] * lw1[noff[dir] + l];
      const double mm = lw1[sown + m];
      z = n + beta * z;
      q = mm + beta * q;
      sv_ = wv + beta * sv_;
      p = u + beta * p;
      x += alpha * p;
      r -= alpha * sv_;
      u -= alpha * q;
      wv -= alpha * z;
      gamma_prev = gamma;
      alpha_prev = alpha;
      __syncthreads();
    }
    if (own) vx[t] = x;
  } else
  for (;; ++it) {
    // dot products of this iteration, the coarse-space restriction of w, and
    // m = B^+ w published for the neighbours
    double gd[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double c6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int e = t; e < nrow; e += COARSE_NT) {
      const double u = vu[e], wv = vw[e];
      gd[0] += vr[e] * u;
      gd[1] += wv * u;
      lown[e] = wv;
      if (two && e % Q < 6) {
        const double* d = ldxy + 3 * (s0 - w0 + e / Q);
        agg_restrict(e % Q, wv, d[0], d[1], c6);
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) gd[2 + k] = c6[k];
    __syncthreads();
    double* mpub = (it & 1) ? A.pub0 : A.pub2;
#pragma unroll 4
    for (int e = t; e < nrow; e += COARSE_NT) {
      const double mv = pinv_row(bi, s0 + e / Q, s0, e % Q, lown);
      if (nwg == 1) lw1[e] = mv;            // one workgroup: the window is its own sets
      else pub_store(&mpub[r0 + e], mv);
    }
    if (!grid_publish_wait<8>(gd, A.red, A.flags, base + (++nsync), slot, ctrl, w, nwg, spin, sslot, sv))
      return;
    // one round trip: the partial sums, the restrictions and the neighbours' m
    grid_collect_window<2, 1, 16>(A.red, slot, nwg, sv, lw1, mpub + (size_t)w0 * Q, win * Q, 2,
                           two ? 1 : 0, A.agg_g, A.naggr, s_c);
    if (two && nwg == 1 && t < 6) s_c[t] = sv[2 + t];
    slot ^= 1;
    __syncthreads();
    const double gamma = sv[0], delta = sv[1];
    if (it == 0) gamma0 = A.coarse_ref ? gamma_zero : gamma;
    if (it >= A.coarse_iters || !(gamma > 0.0) ||
        !(gamma > A.coarse_rtol * A.coarse_rtol * gamma0)) break;
    double alpha, beta;
    if (it == 0) {
      beta = 0.0;
      alpha = delta > 0.0 ? gamma / delta : 0.0;
    } else {
      beta = gamma / gamma_prev;
      const double den = delta - beta * gamma / alpha_prev;
      alpha = den > 0.0 ? gamma / den : 0.0;
    }
    if (!(alpha > 0.0)) break;
    if (two) coarse_space_correction(A, nwa, win, s_c, s_y, lw1, lrows, ldxy, lpart, 6 * alay.nwa_max);
#pragma unroll 1
    for (int e = t; e < nrow; e += COARSE_NT) {
      const double n = coarse_row<kWide>(g, bd, ob, s0 + e / Q, s0, e % Q, lw1, w0);
      const double m = lw1[(size_t)(s0 - w0) * Q + e];
      const double z = n + beta * vz[e];
      const double q = m + beta * vq[e];
      const double sv = vw[e] + beta * vs[e];
      const double p = vu[e] + beta * vp[e];
      vz[e] = z; vq[e] = q; vs[e] = sv; vp[e] = p;
      vx[e] += alpha * p;
      vr[e] -= alpha * sv;
      vu[e] -= alpha * q;
      vw[e] -= alpha * z;
    }
    gamma_prev = gamma;
    alpha_prev = alpha;
    __syncthreads();
  }
  if (A.vec_lds)
    for (int e = t; e < nrow; e += COARSE_NT) A.a[r0 + e] = vx[e];
  if (w == 0 && t == 0) {
    ctrl->coarse_iters += it;
    ctrl->bar_gen = base + nsync;
    ctrl->k = iter + 1;      // every workgroup read k at its start (before the first grid sum)
  }
  // diagnostics: the upper-level system just solved
  if (A.tr_kdiag)
    for (size_t e = (size_t)s0 * Q * Q + t; e < (size_t)s1 * Q * Q; e += COARSE_NT) A.tr_kdiag[e] = A.bdiag[e];
  if (A.tr_koff)
    for (size_t e = (size_t)s0 * NDIR * Q * Q + t; e < (size_t)s1 * NDIR * Q * Q; e += COARSE_NT) A.tr_koff[e] = A.off[e];
  if (A.tr_force)
    for (size_t e = (size_t)s0 * Q + t; e < (size_t)s1 * Q; e += COARSE_NT) A.tr_force[e] = A.force[e];
  if (A.tr_coef)
    for (int e = t; e < nrow; e += COARSE_NT) A.tr_coef[r0 + e] = A.a[r0 + e];
}

__global__ __launch_bounds__(COARSE_NT) void k_coarse(Geo g, CoarseArgs A) {
  coarse_body<true>(g, A, blockIdx.x, gridDim.x);
}

// Fused launch: lattice b owns workgroups [wg0, wg0 + nwg) of the launch and
// runs its own grid sums among them.  A workgroup's place in that order is
// not its blockIdx but a ticket drawn when it starts, so the k-th workgroup
// to start serves launch-wide index k.  The launch may then hold more
// workgroups than fit the device at once: every lattice whose indices were
// all handed out has all of its workgroups running and finishes without
// waiting on anything else, so slots keep freeing until the one lattice
// that is partly started gets the rest of its workgroups.  Workgroups are
// dispatched to the XCDs round-robin by blockIdx, so the rest may all be
// queued on one XCD; that XCD always frees a slot for them only if the
// partly started lattice cannot fill it, so a launch that exceeds the
// device holds lattices of at most one XCD's co-resident workgroups each
// (the caller plans it so).  The workgroup that draws the last ticket resets
// the counter for the next launch on the stream.
// (two workgroups per CU: more lattices' upper levels run at once)
__global__ __launch_bounds__(COARSE_NT, 2) void k_coarse_batch(const BatchEntry* __restrict__ B,
                                                            const int* __restrict__ wg_lat,
                                                            unsigned* __restrict__ ticket) {
  __shared__ int s_gw;
  if (threadIdx.x == 0) {
    const unsigned k = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k + 1 == gridDim.x) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_gw = (int)k;
  }
  __syncthreads();
  const int gw = s_gw;
  const BatchEntry& e = B[wg_lat[gw]];
  coarse_body<false>(e.g, e.ca, gw - e.wg0, e.nwg);
}

// ---------------------------------------------------------------------------
// Coarse space of the upper-level preconditioner, set up once per lattice.
// ---------------------------------------------------------------------------
namespace {
// Entry [m][k] of set s's slice of P0: set mode m (0..5) in aggregate mode k.
__device__ __forceinline__ double agg_p(int m, int k, double dx, double dy) {
  if (m == 0) return k == 0 ? 1.0 : k == 2 ? dx : k == 3 ? dy : 0.0;
  if (m == 1) return k == 1 ? 1.0 : k == 4 ? dx : k == 5 ? dy : 0.0;
  return k == m ? 0.5 : 0.0;
}
}  // namespace

// Block row a of A0 = P0^T K_a P0 from the constant mode 1-6 blocks: the
// set's own block g1 and the 6 x 6 corners of its neighbour blocks.  Thread
// (k, k') < 36 owns entry (k, k') of every 6 x 6 block of the row and adds
// the sets' contributions in a fixed order.
__global__ __launch_bounds__(64) void k_agg_assemble(Geo g, const double* __restrict__ g1,
                                                     const double* __restrict__ off,
                                                     const double* __restrict__ agg_xy,
                                                     int agg_sets, int naggr, double* A0) {
  __shared__ double row[6 * 6 * AGG_MAX];
  const int a = blockIdx.x, t = threadIdx.x, n = 6 * naggr;
  for (int e = t; e < 6 * n; e += 64) row[e] = 0.0;
  __syncthreads();
  if (t < 36) {
    const int k = t / 6, kp = t % 6;
    const int sa = a * agg_sets, sb = min(g.M, sa + agg_sets);
    for (int I = sa; I < sb; ++I) {
      double dxI, dyI;
      agg_coef(g, agg_xy, agg_sets, I, dxI, dyI);
      const int Ii = I % g.mx, Ij = I / g.mx;
      for (int d = -1; d < NDIR; ++d) {
        int J = I;
        if (d >= 0) {
          const int I2 = Ii + nb_di(d), J2 = Ij + nb_dj(d);
          if (I2 < 0 || I2 >= g.mx || J2 < 0 || J2 >= g.my) continue;
          J = J2 * g.mx + I2;
        }
        double dxJ, dyJ;
        agg_coef(g, agg_xy, agg_sets, J, dxJ, dyJ);
        double c = 0.0;
        for (int m = 0; m < 6; ++m) {
          const double pm = agg_p(m, k, dxI, dyI);
          if (pm == 0.0) continue;
          double kl = 0.0;
          for (int l = 0; l < 6; ++l) {
            const double pl = agg_p(l, kp, dxJ, dyJ);
            if (pl == 0.0) continue;
            const double kml = d < 0 ? g1[(size_t)I * 36 + m * 6 + l]
                                     : off[((size_t)I * NDIR + d) * Q * Q + m * Q + l];
            kl += kml * pl;
          }
          c += pm * kl;
        }
        row[k * n + 6 * (J / agg_sets) + kp] += c;
      }
    }
  }
  __syncthreads();
  for (int e = t; e < 6 * n; e += 64) A0[(size_t)(6 * a + e / n) * n + e % n] = row[e];
}

// In place: A0 -> its pseudo-inverse.  Symmetric Jacobi scaling, then
// Gauss-Jordan elimination without row exchanges (A0 is symmetric positive
// semidefinite) that drops a variable whose pivot falls below 1e-9 (it is,
// to that level, a combination of the variables before it), then the
// scaling back and a symmetrisation.  One workgroup.
__global__ __launch_bounds__(1024) void k_agg_invert(double* A, int n) {
  __shared__ double sc[6 * AGG_MAX], rowk[6 * AGG_MAX], colk[6 * AGG_MAX];
  const int t = threadIdx.x, nt = blockDim.x;
  for (int i = t; i < n; i += nt) {
    const double d = A[(size_t)i * n + i];
    sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int e = t; e < n * n; e += nt) A[e] *= sc[e / n] * sc[e % n];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double p = A[(size_t)k * n + k];
    const bool keep = p > 1e-9;
    for (int j = t; j < n; j += nt) {
      rowk[j] = keep ? (j == k ? 1.0 / p : A[(size_t)k * n + j] / p) : 0.0;
      colk[j] = keep && j != k ? A[(size_t)j * n + k] : 0.0;
    }
    __syncthreads();
    for (int e = t; e < n * n; e += nt) {
      const int i = e / n, j = e % n;
      if (!keep) {
        if (i == k || j == k) A[e] = 0.0;
      } else if (i == k) {
        A[e] = rowk[j];
      } else {
        A[e] = (j == k ? 0.0 : A[e]) - colk[i] * rowk[j];
      }
    }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += nt) {
    const int i = e / n, j = e % n;
    if (i <= j) {
      const double v = 0.5 * (A[e] + A[(size_t)j * n + i]) * sc[i] * sc[j];
      A[e] = v;
      A[(size_t)j * n + i] = v;
    }
  }
}

hipError_t launch_agg_setup(const Geo& g, const double* g1, const double* off,
                            const double* agg_xy, int agg_sets, int naggr, double* A0,
                            hipStream_t stream) {
  if (naggr <= 0 || naggr > AGG_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_agg_assemble, dim3(naggr), dim3(64), 0, stream, g, g1, off, agg_xy,
                     agg_sets, naggr, A0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_agg_invert, dim3(1), dim3(1024), 0, stream, A0, 6 * naggr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Create time: constant 6x6 block of the translation/gradient modes,
// G[m][l] = u_hat_m . k^Inner u_hat_l, m, l in 1..6 (Eq. 6 with Eq. 9-10).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_group1(Geo g, const float* __restrict__ ea,
                                                const uint8_t* __restrict__ mask, double* g1) {
  __shared__ double sacc[4][36];
  const int s = blockIdx.x, I = s % g.mx, J = s / g.mx, E = g.E;
  const int i0 = I * E, j0 = J * E, tw = min(E, g.nx - i0), th = min(E, g.ny - j0);
  const size_t plane = (size_t)(g.ny + 2) * g.pitch;
  const double inv_hs = 2.0 / E;
  const int t = threadIdx.x;
  double acc[36];
#pragma unroll
  for (int v = 0; v < 36; ++v) acc[v] = 0.0;
  const int di[6] = {1, -1, 0, 0, -1, 1};
  const int dj[6] = {0, 0, 1, -1, 1, -1};
  const double nvx[6] = {1.0, 1.0, 0.5, 0.5, -0.5, -0.5};
  const double nvy[6] = {0.0, 0.0, kS3, kS3, kS3, kS3};
  for (int n = t; n < tw * th; n += 256) {
    const int ai = i0 + n % tw, aj = j0 + n / tw;
    const size_t pa = pidx(g, ai, aj);
    if (mask[pa]) continue;
    const float kr[6] = {ea[pa], ea[pa - 1], ea[plane + pa], ea[plane + pa - g.pitch],
                         ea[2 * plane + pa], ea[2 * plane + pa - g.pitch + 1]};
    double xa, ya;
    set_coords(ai, aj, i0, j0, tw, th, inv_hs, xa, ya);
    const double ux[6] = {1, 0, xa, ya, 0, 0}, uy[6] = {0, 1, 0, 0, xa, ya};
    double wx[6] = {0, 0, 0, 0, 0, 0}, wy[6] = {0, 0, 0, 0, 0, 0};
    for (int b = 0; b < 6; ++b) {
      const int bi = ai + di[b], bj = aj + dj[b];
      const bool in_set = bi >= i0 && bi < i0 + tw && bj >= j0 && bj < j0 + th &&
                          mask[pidx(g, bi, bj)] == 0;
      double xb, yb;
      set_coords(bi, bj, i0, j0, tw, th, inv_hs, xb, yb);
      const double vx[6] = {1, 0, xb, yb, 0, 0}, vy[6] = {0, 1, 0, 0, xb, yb};
      for (int l = 0; l < 6; ++l) {
        const double dx = ux[l] - (in_set ? vx[l] : 0.0), dy = uy[l] - (in_set ? vy[l] : 0.0);
        const double sv = (double)kr[b] * (nvx[b] * dx + nvy[b] * dy);
        wx[l] += sv * nvx[b];
        wy[l] += sv * nvy[b];
      }
    }
    for (int m = 0; m < 6; ++m)
      for (int l = 0; l < 6; ++l) acc[m * 6 + l] += ux[m] * wx[l] + uy[m] * wy[l];
  }
#pragma unroll
  for (int v = 0; v < 36; ++v) acc[v] = wave_sum(acc[v]);
  if ((t & 63) == 0)
    for (int v = 0; v < 36; ++v) sacc[t >> 6][v] = acc[v];
  __syncthreads();
  if (t < 36) {
    const int m = t / 6, l = t % 6;
    // symmetrise: the two triangles differ only by rounding
    double s1 = 0.0, s2 = 0.0;
    for (int w = 0; w < 4; ++w) { s1 += sacc[w][m * 6 + l]; s2 += sacc[w][l * 6 + m]; }
    g1[(size_t)s * 36 + t] = 0.5 * (s1 + s2);
  }
}

// ---------------------------------------------------------------------------
// Set-up, copy and certification kernels.
// ---------------------------------------------------------------------------
__global__ void k_pad_copy(Geo g, const float* __restrict__ ea_user,
                           const uint8_t* __restrict__ fixed_user, int ea_default,
                           int fixed_default, float* ea, uint8_t* mask, int* stats) {
  const size_t plane = (size_t)(g.ny + 2) * g.pitch;
  const size_t nn = (size_t)g.nx * g.ny;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % g.nx), j = (int)(n / g.nx);
    const size_t p = pidx(g, i, j);
    const bool absent[3] = {i == g.nx - 1, j == g.ny - 1, i == 0 || j == g.ny - 1};
    for (int d = 0; d < 3; ++d) {
      float v = ea_default ? 1.0f : ea_user[(size_t)d * nn + n];
      if (!absent[d] && !(v >= 0.0f && v <= 3.4e38f)) atomicAdd(&stats[0], 1);
      ea[d * plane + p] = absent[d] ? 0.0f : v;
    }
    const uint8_t fx = fixed_default ? (uint8_t)(i == 0) : (uint8_t)(fixed_user[n] != 0);
    mask[p] = fx;
    if (fx) atomicAdd(&stats[1], 1);
    if (!fx) {
      // the free node's own 2 x 2 block, sum of k n n^T over its (up to six)
      // rods; singular when no rod, or only collinear rods, hold the node
      auto rod = [&](int d, int ii, int jj) -> double {
        if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny) return 0.0;
        const bool gone = d == 0 ? ii == g.nx - 1 : d == 1 ? jj == g.ny - 1 : (ii == 0 || jj == g.ny - 1);
        if (gone) return 0.0;
        const double v = ea_default ? 1.0 : (double)ea_user[(size_t)d * nn + (size_t)jj * g.nx + ii];
        return v >= 0.0 && v <= 3.4e38 ? v : 0.0;
      };
      const double ka = rod(0, i, j) + rod(0, i - 1, j);
      const double kb = rod(1, i, j) + rod(1, i, j - 1);
      const double kc = rod(2, i, j) + rod(2, i + 1, j - 1);
      const double dxx = ka + 0.25 * (kb + kc), dyy = 0.75 * (kb + kc), dxy = 0.5 * kS3 * (kb - kc);
      const double tr = dxx + dyy, det = dxx * dyy - dxy * dxy;
      if (!(tr > 0.0) || !(det > 1e-12 * tr * tr)) atomicAdd(&stats[2], 1);
    }
  }
}

template <typename T>
__global__ void k_init_state(Geo g, const uint8_t* __restrict__ mask, const double2* u_fixed,
                             const double2* u_user, int warm, double2* u0, double2* u1,
                             void* d0v, void* d1v, double* a, unsigned* flags, Ctrl* ctrl) {
  using T2 = typename V2<T>::type;
  T2* d0 = reinterpret_cast<T2*>(d0v);
  T2* d1 = reinterpret_cast<T2*>(d1v);
  const size_t nn = (size_t)g.nx * g.ny;
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t nt = (size_t)gridDim.x * blockDim.x;
  for (size_t n = tid; n < nn; n += nt) {
    const int i = (int)(n % g.nx), j = (int)(n / g.nx);
    const size_t p = pidx(g, i, j);
    double2 u = make_double2(0.0, 0.0);
    if (mask[p]) { if (u_fixed) u = u_fixed[n]; }
    else if (warm) u = u_user[n];
    u0[p] = u;
    u1[p] = u;
    d0[p] = mk2<T>((T)0, (T)0);
    d1[p] = mk2<T>((T)0, (T)0);
  }
  for (size_t e = tid; e < (size_t)g.M * Q; e += nt) a[e] = 0.0;
  for (size_t e = tid; e < (size_t)COARSE_MAX_WG; e += nt) flags[e] = 0u;
  if (tid == 0) {
    ctrl->k = 0; ctrl->done = 0; ctrl->status = 0; ctrl->iters = 0; ctrl->err = 0;
    ctrl->coarse_iters = 0; ctrl->r1 = 0.0; ctrl->r2 = 0.0;
    ctrl->bar_count = 0u; ctrl->bar_gen = 0u;
  }
}

__global__ void k_copy_out(Geo g, const double2* __restrict__ u_pad, double2* u_user) {
  const size_t nn = (size_t)g.nx * g.ny;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    u_user[n] = u_pad[pidx(g, (int)(n % g.nx), (int)(n / g.nx))];
  }
}

template <typename T>
__global__ void k_copy_delta(Geo g, const void* d_pad, double2* out) {
  using T2 = typename V2<T>::type;
  const T2* d = reinterpret_cast<const T2*>(d_pad);
  const size_t nn = (size_t)g.nx * g.ny;
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    const T2 v = d[pidx(g, (int)(n % g.nx), (int)(n / g.nx))];
    out[n] = make_double2((double)v.x, (double)v.y);
  }
}

// r = f - K u on unpadded arrays; per-block partials of sum|r|, sum r^2,
// sum|f|, sum f^2 (free DOFs) and the energy 1/2 u.K.u - f.u (Eq. 2).
constexpr int RES_NT = 256;
constexpr int RES_NB_MAX = 4096;
__global__ __launch_bounds__(RES_NT) void k_residual(Geo g, const float* __restrict__ ea,
                                                     const uint8_t* __restrict__ mask,
                                                     const double2* __restrict__ f,
                                                     const double2* __restrict__ u,
                                                     const double2* __restrict__ ufix, double2* r,
                                                     double* partials) {
  __shared__ double sl[RES_NT / 64][5];
  const size_t plane = (size_t)(g.ny + 2) * g.pitch;
  const size_t nn = (size_t)g.nx * g.ny;
  double acc[5] = {0, 0, 0, 0, 0};
  const int di[6] = {1, -1, 0, 0, -1, 1};
  const int dj[6] = {0, 0, 1, -1, 1, -1};
  const double nvx[6] = {1.0, 1.0, 0.5, 0.5, -0.5, -0.5};
  const double nvy[6] = {0.0, 0.0, kS3, kS3, kS3, kS3};
  for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < nn;
       n += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % g.nx), j = (int)(n / g.nx);
    const size_t p = pidx(g, i, j);
    const float kr[6] = {ea[p], ea[p - 1], ea[plane + p], ea[plane + p - g.pitch],
                         ea[2 * plane + p], ea[2 * plane + p - g.pitch + 1]};
    const double2 ua = u[n];
    double kx = 0.0, ky = 0.0, en = 0.0;
    for (int b = 0; b < 6; ++b) {
      const int bi = i + di[b], bj = j + dj[b];
      if (bi < 0 || bi >= g.nx || bj < 0 || bj >= g.ny) continue;
      const double2 ub = u[(size_t)bj * g.nx + bi];
      const double e = nvx[b] * (ua.x - ub.x) + nvy[b] * (ua.y - ub.y);
      const double s = (double)kr[b] * e;
      kx += s * nvx[b];
      ky += s * nvy[b];
      en += 0.25 * s * e;        // each rod is seen from both ends
    }
    double2 rv = make_double2(0.0, 0.0);
    if (!mask[p]) {
      const double2 fv = f[n];
      rv = make_double2(fv.x - kx, fv.y - ky);
      double2 rhs = fv;
      if (ufix) {
        // f - K_fc u_c: rods ending on clamped nodes pull with k n (n . u_c)
        for (int b = 0; b < 6; ++b) {
          const int bi = i + di[b], bj = j + dj[b];
          if (bi < 0 || bi >= g.nx || bj < 0 || bj >= g.ny) continue;
          if (!mask[pidx(g, bi, bj)]) continue;
          const double2 ub = ufix[(size_t)bj * g.nx + bi];
          const double sv = (double)kr[b] * (nvx[b] * ub.x + nvy[b] * ub.y);
          rhs.x += sv * nvx[b];
          rhs.y += sv * nvy[b];
        }
      }
      acc[0] += fabs(rv.x) + fabs(rv.y);
      acc[1] += rv.x * rv.x + rv.y * rv.y;
      acc[2] += fabs(rhs.x) + fabs(rhs.y);
      acc[3] += rhs.x * rhs.x + rhs.y * rhs.y;
      en -= fv.x * ua.x + fv.y * ua.y;
    }
    acc[4] += en;
    if (r) r[n] = rv;
  }
  for (int v = 0; v < 5; ++v) acc[v] = wave_sum(acc[v]);
  if ((threadIdx.x & 63) == 0)
    for (int v = 0; v < 5; ++v) sl[threadIdx.x >> 6][v] = acc[v];
  __syncthreads();
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int w = 0; w < RES_NT / 64; ++w) s += sl[w][threadIdx.x];
    partials[(size_t)blockIdx.x * 5 + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(RES_NT) void k_reduce5(const double* partials, int nb, double* out) {
  __shared__ double sl[RES_NT / 64][5];
  double acc[5] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += RES_NT)
    for (int v = 0; v < 5; ++v) acc[v] += partials[(size_t)b * 5 + v];
  for (int v = 0; v < 5; ++v) acc[v] = wave_sum(acc[v]);
  if ((threadIdx.x & 63) == 0)
    for (int v = 0; v < 5; ++v) sl[threadIdx.x >> 6][v] = acc[v];
  __syncthreads();
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int w = 0; w < RES_NT / 64; ++w) s += sl[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
namespace {
int grid_for(size_t n, int nt, int cap) {
  size_t b = (n + nt - 1) / nt;
  if (b < 1) b = 1;
  return (int)(b > (size_t)cap ? cap : b);
}
}  // namespace

// Threads per tile workgroup for each set edge, precision and overlap
// (measured without overlap: 256 for E = 32; 512 for E = 64 in float32, 1024
// in float64, where 512 threads spill).  With overlap the region holds
// (E + 2 OV)^2 nodes: 256 threads for E = 16; for 64, 512 in float32 (ten
// or eleven nodes per thread in 256 registers; at 4096^2 1.20x faster than
// 1024 threads at 128 with overlap 2, 1.38x with overlap 4) and 1024 in
// float64 (1.28x faster than 512 with overlap 2, 1.09x with 4); for 32, 512 (three nodes per
// thread; in float64 256 or 1024 threads were 1.3x slower; in float32 256
// threads, two tiles per CU without spills, were 1.02-1.07x faster on single
// lattices from 1024^2 up but 1.02x slower in fused batches and served
// streams of small lattices).  The choice depends on the lattice's set edge,
// form and overlap only, so a lattice gets the same kernel alone and in a
// fused batch.  TL_TILE_THREADS overrides for tuning.
static int tile_threads(int E, bool mixed, int ov) {
  const char* v = getenv("TL_TILE_THREADS");
  const int env = v && *v ? atoi(v) : 0;
  if (E == 16) return 256;
  if (ov > 0) {
    if (E == 32) return env == 256 || env == 512 ? env : 512;
    return env == 512 || env == 1024 ? env : (mixed ? 512 : 1024);
  }
  if (E == 32) return env == 256 || env == 512 || env == 1024 ? env : 256;
  return env == 512 || env == 1024 ? env : (mixed ? 512 : 1024);
}

bool tile_overlap_supported(int ov) { return ov == 0 || ov == 1 || ov == 2 || ov == 4; }

// Instantiations: (set edge, threads) for every overlap, float and double.
#define TL_TILE_SHAPES(X, T, OV)                                   \
  if (E == 16) X(T, 16, 256, OV);                                  \
  else if (E == 32 && nt == 256) X(T, 32, 256, OV);                \
  else if (E == 32 && nt == 512) X(T, 32, 512, OV);                \
  else if (E == 32 && OV == 0) X(T, 32, 1024, 0);                  \
  else if (E == 64 && nt == 512) X(T, 64, 512, OV);                \
  else if (E == 64) X(T, 64, 1024, OV);                            \
  else return hipErrorInvalidValue;
#define TL_TILE_OVERLAPS(X, T)                 \
  if (ov == 0) { TL_TILE_SHAPES(X, T, 0) }     \
  else if (ov == 1) { TL_TILE_SHAPES(X, T, 1) } \
  else if (ov == 2) { TL_TILE_SHAPES(X, T, 2) } \
  else if (ov == 4) { TL_TILE_SHAPES(X, T, 4) } \
  else return hipErrorInvalidValue;

hipError_t launch_tile(bool mixed, int ov, const Geo& g, const float* ea, const uint8_t* mask,
                       const TileArgs& a, hipStream_t stream) {
  const dim3 grid(g.M);
  const int E = g.E;
  const int nt = tile_threads(E, mixed, ov);
  const size_t dyn = a.band ? band_chunk_bytes(E + 2 * ov) : 0;
#define TL_TILE(T, EE, NT, OV)                                                                     \
  do {                                                                                             \
    if (dyn && hipFuncSetAttribute((const void*)k_tile<T, EE, NT, OV>,                             \
                                   hipFuncAttributeMaxDynamicSharedMemorySize,                     \
                                   (int)dyn) != hipSuccess)                                        \
      return hipErrorInvalidValue;                                                                 \
    hipLaunchKernelGGL((k_tile<T, EE, NT, OV>), grid, dim3(NT), dyn, stream, g, ea, mask, a);      \
  } while (0)
  if (mixed) {
    TL_TILE_OVERLAPS(TL_TILE, float)
  } else {
    TL_TILE_OVERLAPS(TL_TILE, double)
  }
#undef TL_TILE
  return hipGetLastError();
}

hipError_t launch_tile_batch(bool mixed, int E, int ov, const BatchEntry* B, const int* tile_lat,
                             int ntiles, bool any_band, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 grid(ntiles);
  const int nt = tile_threads(E, mixed, ov);
  const size_t dyn = any_band ? band_chunk_bytes(E + 2 * ov) : 0;
#define TL_TILEB(T, EE, NT, OV)                                                                    \
  do {                                                                                             \
    if (dyn && hipFuncSetAttribute((const void*)k_tile_batch<T, EE, NT, OV>,                       \
                                   hipFuncAttributeMaxDynamicSharedMemorySize,                     \
                                   (int)dyn) != hipSuccess)                                        \
      return hipErrorInvalidValue;                                                                 \
    hipLaunchKernelGGL((k_tile_batch<T, EE, NT, OV>), grid, dim3(NT), dyn, stream, B, tile_lat);   \
  } while (0)
  if (mixed) {
    TL_TILE_OVERLAPS(TL_TILEB, float)
  } else {
    TL_TILE_OVERLAPS(TL_TILEB, double)
  }
#undef TL_TILEB
  return hipGetLastError();
}
#undef TL_TILE_OVERLAPS
#undef TL_TILE_SHAPES

hipError_t launch_offdiag_batch(bool mixed, const BatchEntry* B, const int* set_lat, int nsets,
                                hipStream_t stream) {
  if (nsets <= 0) return hipSuccess;
  if (mixed) hipLaunchKernelGGL(k_offdiag_batch<float>, dim3(nsets), dim3(256), 0, stream, B, set_lat);
  else hipLaunchKernelGGL(k_offdiag_batch<double>, dim3(nsets), dim3(256), 0, stream, B, set_lat);
  return hipGetLastError();
}

hipError_t launch_blockinv_batch(const BatchEntry* B, const int* set_lat, int nsets,
                                 hipStream_t stream) {
  if (nsets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_blockinv_batch, dim3((nsets + BLOCKINV_SETS - 1) / BLOCKINV_SETS), dim3(64), 0,
                     stream, B, set_lat, nsets);
  return hipGetLastError();
}

// Co-resident workgroups of the fused upper-level kernel at `lds` bytes of
// dynamic LDS: the occupancy per CU times the CUs, or at most the value of
// TL_COARSE_BATCH_WG when set (for runs under tools that can keep part of the
// device from a kernel, such as hardware counter collection; a lattice's own
// workgroup count and with it its results do not change).  With the cap set,
// coarse_batch_oversubscribe() is false: every launch's workgroups must then
// fit the cap at once.
int coarse_batch_capacity(size_t lds) {
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)k_coarse_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                            COARSE_DYN_LDS_MAX) != hipSuccess)
      return 0;
    attr_set = true;
  }
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_coarse_batch, COARSE_NT,
                                                   lds) != hipSuccess)
    return 0;
  int cap = per_cu * cus;
  const char* v = getenv("TL_COARSE_BATCH_WG");
  if (v && *v && atoi(v) > 0) cap = std::min(cap, atoi(v));
  return cap;
}

bool coarse_batch_oversubscribe() {
  const char* v = getenv("TL_COARSE_BATCH_WG");
  return !(v && *v && atoi(v) > 0);
}

hipError_t launch_coarse_batch(const BatchEntry* B, const int* wg_lat, unsigned* ticket, int nwg,
                               int max_lattice_nwg, size_t lds, hipStream_t stream) {
  if (nwg <= 0) return hipSuccess;
  if (coarse_batch_capacity(lds) < max_lattice_nwg) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_coarse_batch, dim3(nwg), dim3(COARSE_NT), lds, stream, B, wg_lat, ticket);
  return hipGetLastError();
}

__global__ void k_gather_ctrl(const BatchEntry* __restrict__ B, int n, Ctrl* out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) out[b] = *B[b].ca.ctrl;
}

hipError_t launch_gather_ctrl(const BatchEntry* B, int n, Ctrl* out, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_ctrl, dim3((n + 63) / 64), dim3(64), 0, stream, B, n, out);
  return hipGetLastError();
}

hipError_t launch_offdiag(bool mixed, const Geo& g, const float* ea, const uint8_t* mask,
                          const OffArgs& a, hipStream_t stream) {
  if (mixed) hipLaunchKernelGGL(k_offdiag<float>, dim3(g.M), dim3(256), 0, stream, g, ea, mask, a);
  else hipLaunchKernelGGL(k_offdiag<double>, dim3(g.M), dim3(256), 0, stream, g, ea, mask, a);
  return hipGetLastError();
}

hipError_t launch_blockinv(const Geo& g, const BlockArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(k_blockinv, dim3((g.M + BLOCKINV_SETS - 1) / BLOCKINV_SETS), dim3(64), 0, stream, g, a);
  return hipGetLastError();
}

hipError_t launch_coarse(const Geo& g, const CoarseArgs& a, hipStream_t stream) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_coarse,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, COARSE_DYN_LDS_MAX);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const size_t lds = coarse_lds_bytes(g, a.nwg, a.vec_lds, a.blk_lds, a.naggr > 0);
  if (lds > COARSE_DYN_LDS_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_coarse, dim3(a.nwg), dim3(COARSE_NT), lds, stream, g, a);
  return hipGetLastError();
}

hipError_t launch_band_factor(const Geo& g, int ov, const float* ea, const uint8_t* mask,
                              double* band, hipStream_t stream) {
  const int R = g.E + 2 * ov;
  const size_t lds = (size_t)(2 * R + 2) * band_bs(R) * sizeof(double);   // b_max + 1 columns
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_band_factor, dim3(g.M), dim3(256), lds, stream, g, ov, ea, mask, band);
  return hipGetLastError();
}

hipError_t launch_group1(const Geo& g, const float* ea, const uint8_t* mask, double* g1,
                         hipStream_t stream) {
  hipLaunchKernelGGL(k_group1, dim3(g.M), dim3(256), 0, stream, g, ea, mask, g1);
  return hipGetLastError();
}

hipError_t launch_init_state(const Geo& g, const uint8_t* mask, const double2* u_fixed,
                             const double2* u_user, int warm, double2* u0, double2* u1,
                             void* d0, void* d1, bool mixed, double* a, unsigned* flags,
                             Ctrl* ctrl, hipStream_t stream) {
  const int nb = grid_for((size_t)g.nx * g.ny, 256, 8192);
  if (mixed)
    hipLaunchKernelGGL(k_init_state<float>, dim3(nb), dim3(256), 0, stream, g, mask, u_fixed,
                       u_user, warm, u0, u1, d0, d1, a, flags, ctrl);
  else
    hipLaunchKernelGGL(k_init_state<double>, dim3(nb), dim3(256), 0, stream, g, mask, u_fixed,
                       u_user, warm, u0, u1, d0, d1, a, flags, ctrl);
  return hipGetLastError();
}

hipError_t launch_copy_out(const Geo& g, const double2* u_pad, double2* u_user,
                           hipStream_t stream) {
  const int nb = grid_for((size_t)g.nx * g.ny, 256, 8192);
  hipLaunchKernelGGL(k_copy_out, dim3(nb), dim3(256), 0, stream, g, u_pad, u_user);
  return hipGetLastError();
}

hipError_t launch_copy_delta(bool mixed, const Geo& g, const void* d_pad, double2* out,
                             hipStream_t stream) {
  const int nb = grid_for((size_t)g.nx * g.ny, 256, 8192);
  if (mixed) hipLaunchKernelGGL(k_copy_delta<float>, dim3(nb), dim3(256), 0, stream, g, d_pad, out);
  else hipLaunchKernelGGL(k_copy_delta<double>, dim3(nb), dim3(256), 0, stream, g, d_pad, out);
  return hipGetLastError();
}

size_t residual_partials(const Geo& g) {
  return (size_t)grid_for((size_t)g.nx * g.ny, RES_NT, RES_NB_MAX) * 5;
}

hipError_t launch_residual(const Geo& g, const float* ea, const uint8_t* mask,
                           const double2* f, const double2* u, const double2* ufix, double2* r,
                           double* partials, double* out5, hipStream_t stream) {
  const int nb = grid_for((size_t)g.nx * g.ny, RES_NT, RES_NB_MAX);
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(RES_NT), 0, stream, g, ea, mask, f, u, ufix, r, partials);
  hipLaunchKernelGGL(k_reduce5, dim3(1), dim3(RES_NT), 0, stream, partials, nb, out5);
  return hipGetLastError();
}

hipError_t launch_pad_copy_stats(const Geo& g, const float* ea_user, const uint8_t* fixed_user,
                                 int ea_default, int fixed_default, float* ea, uint8_t* mask,
                                 int* stats, hipStream_t stream) {
  const int nb = grid_for((size_t)g.nx * g.ny, 256, 8192);
  hipLaunchKernelGGL(k_pad_copy, dim3(nb), dim3(256), 0, stream, g, ea_user, fixed_user,
                     ea_default, fixed_default, ea, mask, stats);
  return hipGetLastError();
}

}  // namespace tl
