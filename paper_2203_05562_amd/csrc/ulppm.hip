// ulppm.hip -- gfx950 kernels and C ABI for the per-step bond loop of updated
// Lagrangian unsaturated periporomechanics (Menon & Song, arXiv 2203.05562).
//
// One explicit central-difference step (Algorithm 2 driving Algorithm 1):
//   k_predict   velocity predictor, boundary conditions, Kahan-compensated
//               displacement, positions (Eqs. 60-61, 64)
//   families    Verlet candidates within delta plus a skin, rebuilt from a
//               cell list only when a point has moved half the skin
//               (k_check_skin, k_family, k_cand_rev); every step k_filter
//               applies the exact FP64 distance predicate to the candidates,
//               a scan turns the counts into CSR rows and k_compact writes
//               the columns and rev[] through the reverse candidate index
//               (Eq. 1; Algorithm 1, neighbour search)
//   k_point_kin_quad  four lanes per point: full-horizon sums, volume change,
//               porosity, saturation and mass (Eqs. 5, 8, 15-17, 48)
//   k_bond_mx   one workgroup per point i, its family staged in LDS: pass 1
//               forms the sub-horizon sums (shape tensor, velocity-gradient
//               numerator, volume; Eqs. 22-23, 25, 55, 57) as the 0/1
//               membership matrix times a feature matrix on the matrix cores,
//               membership decided by the exact FP64 predicate; the tail (one
//               lane per bond) inverts K_ij in FP64, forms the strain
//               increment, runs the Perzyna return map (Section 3.2.1) and
//               the bond's factor M_j; pass 2 sums the M_j of the sub-horizons
//               holding each member into the force states T_ij (Eqs. 27, 31-32,
//               35; Eqs. 51, 53 as an option); the point history is the
//               volume-weighted mean of the bond states.
//   k_gather    one wave per point: f_i = sum_j (T_ij - T_ji) V_i V_j through
//               rev[] (no atomics), contact with a rigid substrate (Eqs.
//               91-93), acceleration, velocity corrector, energy partials
//               (Eqs. 49-50, 62-63, 66-68)
// The standard correspondence model (Eqs. 12-14) replaces the bond kernel by
// k_point_kin_standard; the history carried on the bonds adds k_hist_map
// and k_hist_keep around it; the k_adj_* kernels run the reverse mode of a
// step (with the bond history, k_hist_carry and k_adj_hist_carry).
//
// Every kernel is stream-ordered on the context's stream.  No kernel traps;
// failures raise device counters.  Memory: all scratch is allocated at
// create; the state lives in caller-owned SoA device arrays.

#include <hip/hip_runtime.h>
#include <functional>
#include <mutex>
#include <type_traits>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/ulppm.h"

namespace {

#ifndef ULPPM_BOND_THREADS
#define ULPPM_BOND_THREADS 128
#endif
#ifndef ULPPM_ADJ_MIN_WAVES
#define ULPPM_ADJ_MIN_WAVES 2
#endif
constexpr int kBondThreads = ULPPM_BOND_THREADS;   // one workgroup per point, one lane per bond
constexpr int kBondWaves = kBondThreads / 64;
constexpr int kWave = 64;
constexpr int kScanChunk = 2048;    // elements per block in the scans (256 x 8)
// Regions of the reduction-partials buffer (doubles).
constexpr int64_t kPartPred = 0;        // predictor energy partials, 2 x <= 2048 blocks
constexpr int64_t kPartRed = 4096;      // bounding box (6 x <= 1024) or dt_crit (<= 1024)
constexpr int64_t kPartGather = 10240;  // gather energy partials, 3 per block

// Device counters, zeroed at the start of every API call.
enum Ctr {
  C_DEGEN = 0, C_PLASTIC, C_MAXNEWTON, C_NOCONV, C_TESTS, C_TRIPLES, C_OVERFLOW,
  C_NONFINITE, C_MAXFAM, C_BONDSUM, C_REBUILD, C_ADJLDS, C_NCOUNT = 16
};
constexpr int kStripes = 256;       // each device counter is striped over this many addresses
constexpr int kTimedSteps = 256;    // steps per call covered by phase timings
constexpr double kSkin = 0.1;       // candidate-list skin, as a fraction of delta
constexpr int kPhases = 5;          // predict, family, bond, gather, point kinematics

struct DevParams {
  double delta, d2;
  double K, mu, M, lam, kap, eta, b1, b2;
  double rho_s, rho_w, a1, a2, n_vg;
  double g0, g1, g2;
  double dt;
  double newton_tol;
  int newton_maxit;
  int force_mode;
  double iM2;                 // 1 / M^2
  int plane;                  // 1: plane strain in the x-z plane, unit thickness
};

struct Grid {                 // cell grid over the current bounding box
  double lo0, lo1, lo2, cs;
  int64_t d0, d1, d2, ncell;
};

// Substrate of the contact model, as the kernels read it.
struct ContactDev {
  double cs, mu_f, dc, dc2, ox, oy, oz, h, Vs;
  int32_t nx, ny, nz, on;
};

// Inclusive index range of lattice sites whose coordinate lies within
// (t_lo, t_hi) in units of the spacing, widened by one site on each side and
// clipped to [0, n); empty when lo > hi.
__device__ __forceinline__ void site_range(double t_lo, double t_hi, int n, int* lo, int* hi) {
  const double a = floor(t_lo) - 1.0, b = ceil(t_hi) + 1.0;
  if (!(b >= 0.0) || !(a <= (double)(n - 1))) { *lo = 0; *hi = -1; return; }
  *lo = a < 0.0 ? 0 : (int)a;
  *hi = b > (double)(n - 1) ? n - 1 : (int)b;
}

// Contact force density on point i from the substrate sites within delta_c
// (Eqs. 91-93): sum_s 2 (T_c + T_f) V_s with T_c = -C_s (delta_c - |Y|) Y/|Y|,
// T_f = -mu_f sign(d|Y|/dt) T_c, Y = x_s - x_i, d|Y|/dt = -Y.v_i/|Y|.  Lanes
// take the sites of the candidate box; the caller reduces over the wave.
__device__ void contact_density(const ContactDev& C, bool plane, double xi, double yi, double zi, double vx,
                                double vy, double vz, int lane, double* out) {
#pragma clang fp contract(off)
  out[0] = out[1] = out[2] = 0.0;
  const double Vs = plane ? C.h * C.h : C.Vs;                  // unit thickness in plane strain
  int a0, a1, b0, b1, k0, k1;
  site_range((xi - C.dc - C.ox) / C.h, (xi + C.dc - C.ox) / C.h, C.nx, &a0, &a1);
  site_range((yi - C.dc - C.oy) / C.h, (yi + C.dc - C.oy) / C.h, C.ny, &b0, &b1);
  site_range((C.oz - zi - C.dc) / C.h, (C.oz - zi + C.dc) / C.h, C.nz, &k0, &k1);
  if (a1 < a0 || b1 < b0 || k1 < k0) return;
  const int na = a1 - a0 + 1, nb = b1 - b0 + 1;
  const int64_t total = (int64_t)na * nb * (k1 - k0 + 1);
  for (int64_t e = lane; e < total; e += kWave) {
    const int a = a0 + (int)(e % na), b = b0 + (int)((e / na) % nb), k = k0 + (int)(e / ((int64_t)na * nb));
    const double Y0 = (C.ox + (double)a * C.h) - xi;
    const double Y1 = (C.oy + (double)b * C.h) - yi;
    const double Y2 = (C.oz - (double)k * C.h) - zi;
    const double r2 = (Y0 * Y0 + Y1 * Y1) + Y2 * Y2;
    if (!(r2 < C.dc2) || r2 == 0.0) continue;
    const double r = sqrt(r2);
    const double tc = -C.cs * (C.dc - r) / r;                  // T_c = tc Y
    const double rate = -(Y0 * vx + Y1 * vy + Y2 * vz);         // |Y| d|Y|/dt
    const double sg = rate > 0.0 ? 1.0 : (rate < 0.0 ? -1.0 : 0.0);
    const double w = 2.0 * Vs * tc * (1.0 - C.mu_f * sg);      // 2 (T_c + T_f) V_s = w Y
    out[0] += w * Y0;
    out[1] += w * Y1;
    out[2] += w * Y2;
  }
}

// Reverse of the contact force of point i (frictional branch frozen):
// with f_i = V_i sum_s c(r) Y, c = -2 V_s (1 - mu_f sg) C_s (delta_c - r)/r
// and Y = x_s - x_i, the adjoint fbar of f_i adds
//   xbar_i -= V_i sum_s [c fbar + (dc/dr)/r (Y . fbar) Y],  dc/dr = 2 V_s (1 - mu_f sg) C_s delta_c / r^2,
//   Vbar_i += sum_s c (Y . fbar).
// Lanes take the sites of the candidate box; the caller reduces over the wave.
__device__ void contact_adjoint(const ContactDev& C, bool plane, double xi, double yi, double zi, double vx,
                                double vy, double vz, double Vi, const double* fb, int lane, double* xbar,
                                double* Vbar) {
#pragma clang fp contract(off)
  xbar[0] = xbar[1] = xbar[2] = 0.0;
  *Vbar = 0.0;
  const double Vs = plane ? C.h * C.h : C.Vs;
  int a0, a1, b0, b1, k0, k1;
  site_range((xi - C.dc - C.ox) / C.h, (xi + C.dc - C.ox) / C.h, C.nx, &a0, &a1);
  site_range((yi - C.dc - C.oy) / C.h, (yi + C.dc - C.oy) / C.h, C.ny, &b0, &b1);
  site_range((C.oz - zi - C.dc) / C.h, (C.oz - zi + C.dc) / C.h, C.nz, &k0, &k1);
  if (a1 < a0 || b1 < b0 || k1 < k0) return;
  const int na = a1 - a0 + 1, nb = b1 - b0 + 1;
  const int64_t total = (int64_t)na * nb * (k1 - k0 + 1);
  for (int64_t e = lane; e < total; e += kWave) {
    const int a = a0 + (int)(e % na), b = b0 + (int)((e / na) % nb), k = k0 + (int)(e / ((int64_t)na * nb));
    const double Y0 = (C.ox + (double)a * C.h) - xi;
    const double Y1 = (C.oy + (double)b * C.h) - yi;
    const double Y2 = (C.oz - (double)k * C.h) - zi;
    const double r2 = (Y0 * Y0 + Y1 * Y1) + Y2 * Y2;
    if (!(r2 < C.dc2) || r2 == 0.0) continue;
    const double r = sqrt(r2);
    const double rate = -(Y0 * vx + Y1 * vy + Y2 * vz);
    const double sg = rate > 0.0 ? 1.0 : (rate < 0.0 ? -1.0 : 0.0);
    const double k2 = 2.0 * Vs * (1.0 - C.mu_f * sg) * C.cs;
    const double c = -k2 * (C.dc - r) / r;
    const double dcr = k2 * C.dc / (r2 * r);                    // (dc/dr) / r
    const double yf = Y0 * fb[0] + Y1 * fb[1] + Y2 * fb[2];
    xbar[0] -= Vi * (c * fb[0] + dcr * yf * Y0);
    xbar[1] -= Vi * (c * fb[1] + dcr * yf * Y1);
    xbar[2] -= Vi * (c * fb[2] + dcr * yf * Y2);
    *Vbar += c * yf;
  }
}

// Device counters are striped by block so that concurrent blocks rarely hit
// the same address; k_reduce_counters folds the stripes once per call.
__device__ __forceinline__ void ctr_add(unsigned long long* ctr, int k, unsigned long long v) {
  atomicAdd(&ctr[k * kStripes + (blockIdx.x & (kStripes - 1))], v);
}
__device__ __forceinline__ void ctr_max(unsigned long long* ctr, int k, unsigned long long v) {
  atomicMax(&ctr[k * kStripes + (blockIdx.x & (kStripes - 1))], v);
}

// Blocks are dispatched round-robin over the 8 XCDs of the chip, each with
// its own L2.  Give each XCD a contiguous range of points so that the
// neighbour data a block gathers is mostly resident in that XCD's L2.
// The grid is launched with 8*per blocks; ids >= n are idle.
__device__ __forceinline__ int64_t xcd_point(int64_t b, int64_t per) {
  return (b & 7) * per + (b >> 3);
}

// Points walked by one wave of a capped grid (a multiple of 8 blocks of
// `wpb` waves): the waves of XCD x stride over that XCD's contiguous range.
// Short per-point kernels use this so that the number of workgroups stays
// small: their run time would otherwise be set by workgroup dispatch.
struct XcdWalk {
  int64_t first, stride, end;
};
// The same walk over groups of lanes: gpb groups per block, g this thread's.
__device__ __forceinline__ XcdWalk xcd_walk_groups(int64_t n, int gpb, int g) {
  const int64_t per = (n + 7) / 8;
  const int64_t x = blockIdx.x & 7, lb = blockIdx.x >> 3, nblk = gridDim.x >> 3;
  XcdWalk w;
  w.first = x * per + lb * gpb + g;
  w.stride = nblk * gpb;
  w.end = (x + 1) * per < n ? (x + 1) * per : n;
  return w;
}
__device__ __forceinline__ XcdWalk xcd_walk(int64_t n, int wpb) {
  const int64_t per = (n + 7) / 8;
  const int64_t x = blockIdx.x & 7, lb = blockIdx.x >> 3, nblk = gridDim.x >> 3;
  XcdWalk w;
  w.first = x * per + lb * wpb + threadIdx.x / kWave;
  w.stride = nblk * wpb;
  w.end = (x + 1) * per < n ? (x + 1) * per : n;
  return w;
}

// Wave reductions with DPP lane exchanges (no LDS traffic): butterflies
// within each row of 16 lanes (quad_perm xor 1 and 2, half-row and row
// mirrors), then row_bcast15 and row_bcast31 carry the row totals into the
// last row; lane 63 holds the wave's total, which is read back uniformly.
template <int Ctrl, int RowMask>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, Ctrl, RowMask, 0xF, false);
}
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<Ctrl, RowMask>((int)b);
  const int hi = dpp_i<Ctrl, RowMask>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int Ctrl, int RowMask>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<Ctrl, RowMask>(__float_as_int(v)));
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140,
              kDppBcast15 = 0x142, kDppBcast31 = 0x143;

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kDppXor1, 0xF>(v);
  v += dpp_d<kDppXor2, 0xF>(v);
  v += dpp_d<kDppHalfMirror, 0xF>(v);
  v += dpp_d<kDppMirror, 0xF>(v);
  v += dpp_d<kDppBcast15, 0xA>(v);
  v += dpp_d<kDppBcast31, 0xC>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<kDppXor1, 0xF>(v);
  v += dpp_f<kDppXor2, 0xF>(v);
  v += dpp_f<kDppHalfMirror, 0xF>(v);
  v += dpp_f<kDppMirror, 0xF>(v);
  v += dpp_f<kDppBcast15, 0xA>(v);
  v += dpp_f<kDppBcast31, 0xC>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ int wave_sum_i(int v) {
  v += dpp_i<kDppXor1, 0xF>(v);
  v += dpp_i<kDppXor2, 0xF>(v);
  v += dpp_i<kDppHalfMirror, 0xF>(v);
  v += dpp_i<kDppMirror, 0xF>(v);
  v += dpp_i<kDppBcast15, 0xA>(v);
  v += dpp_i<kDppBcast31, 0xC>(v);
  return __builtin_amdgcn_readlane(v, 63);
}

// maximum of non-negative values (masked rows contribute 0)
__device__ __forceinline__ int wave_max_i(int v) {
  v = max(v, dpp_i<kDppXor1, 0xF>(v));
  v = max(v, dpp_i<kDppXor2, 0xF>(v));
  v = max(v, dpp_i<kDppHalfMirror, 0xF>(v));
  v = max(v, dpp_i<kDppMirror, 0xF>(v));
  v = max(v, dpp_i<kDppBcast15, 0xA>(v));
  v = max(v, dpp_i<kDppBcast31, 0xC>(v));
  return __builtin_amdgcn_readlane(v, 63);
}

// Exact squared distance, rounded as ((dx^2 + dy^2) + dz^2) with no fused
// multiply-add, compared with delta^2.  Decides family (Eq. 1) and
// sub-horizon (Eq. 22) membership identically on every device.
__device__ __forceinline__ bool within(double ax, double ay, double az, double bx, double by,
                                       double bz, double d2) {
#pragma clang fp contract(off)
  double dx = bx - ax, dy = by - ay, dz = bz - az;
  double r2 = (dx * dx + dy * dy) + dz * dz;
  return r2 <= d2;
}

__device__ __forceinline__ double exact_r2(double ax, double ay, double az, double bx, double by,
                                           double bz) {
#pragma clang fp contract(off)
  double dx = bx - ax, dy = by - ay, dz = bz - az;
  return (dx * dx + dy * dy) + dz * dz;
}

// ---------------------------------------------------------------- scans --
// Exclusive prefix sum of int32 counts into int64 offsets; out[n] = total.

__global__ void k_scan_blocks(const int32_t* __restrict__ cnt, int64_t n, int64_t* __restrict__ out,
                              int64_t* __restrict__ bsum, const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int64_t s[256];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  int64_t loc[8];
  int64_t acc = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int64_t e = base + threadIdx.x * 8 + k;
    int64_t c = e < n ? (int64_t)cnt[e] : 0;
    loc[k] = acc;
    acc += c;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int64_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t pre = threadIdx.x ? s[threadIdx.x - 1] : 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int64_t e = base + threadIdx.x * 8 + k;
    if (e < n) out[e] = pre + loc[k];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = s[255];
}

__global__ void k_scan_top(int64_t* __restrict__ bsum, int64_t nb, int64_t* __restrict__ out, int64_t n,
                           const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  __shared__ int64_t s[1024];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += 1024) {
    int64_t e = base + threadIdx.x;
    int64_t v = e < nb ? bsum[e] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      int64_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (e < nb) bsum[e] = carry + s[threadIdx.x] - v;   // exclusive block offset
    int64_t tot = s[1023];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ boff,
                           const int32_t* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  const int64_t add = boff[blockIdx.x];
  for (int k = threadIdx.x; k < kScanChunk; k += blockDim.x) {
    int64_t e = base + k;
    if (e < n) out[e] += add;
  }
}

template <class T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v, const int32_t* __restrict__ gate = nullptr) {
  if (gate && *gate == 0) return;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

// ------------------------------------------------------------ predictor --

// Velocity predictor v_half = v + (dt/2) a (Eq. 60, beta1 = 1/2, with the step
// size restored); boundary conditions: fixed points (code 1) v_half = 0,
// driven points (code 2) v_half = v, the velocity they keep; displacement
// u += dt v_half (Eqs. 61/64 with beta2 = 0) with Kahan compensation, and
// positions x = x0 + u.  Rounded exactly as written (no contraction), so a
// state gives bit-identical positions on every device.  Also saves V^n and
// the first half of the energy increments (old force f^n = M (a - g)).
__global__ void k_predict(ulppm_state S, DevParams P, double* __restrict__ x, double* __restrict__ vh,
                          double* __restrict__ vol_n, double* __restrict__ epart) {
#pragma clang fp contract(off)
  const int64_t n = S.n;
  const double dt = P.dt, hdt = 0.5 * P.dt;
  const double g[3] = {P.g0, P.g1, P.g2};
  double eint = 0.0, eext = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const bool fx = S.fixed[i] != 0;
    const bool drv = S.fixed[i] == 2;
    const double m = S.mass[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double a = S.a[c][i];
      const double vhalf = drv ? S.v[c][i] : fx ? 0.0 : S.v[c][i] + hdt * a;
      vh[c * n + i] = vhalf;
      const double u = S.u[c][i], uc = S.uc[c][i];
      const double y = dt * vhalf - uc;
      const double t = u + y;
      S.uc[c][i] = (t - u) - y;
      S.u[c][i] = t;
      x[c * n + i] = S.x0[c][i] + t;
      if (!fx) {
        eint -= hdt * vhalf * (m * (a - g[c]));
        eext += hdt * vhalf * m * g[c];
      }
    }
    vol_n[i] = S.vol[i];
  }
  __shared__ double r[2][4];
  eint = wave_sum(eint);
  eext = wave_sum(eext);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) { r[0][w] = eint; r[1][w] = eext; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) { a0 += r[0][k]; a1 += r[1][k]; }
    epart[2 * blockIdx.x] = a0;
    epart[2 * blockIdx.x + 1] = a1;
  }
}

// Positions x = x0 + u without stepping (ulppm_forces, families, dt_crit, init).
__global__ void k_positions(ulppm_state S, double* __restrict__ x, double* __restrict__ vh,
                            double* __restrict__ vol_n) {
  const int64_t n = S.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c * n + i] = S.x0[c][i] + S.u[c][i];
      vh[c * n + i] = S.v[c][i];
    }
    vol_n[i] = S.vol[i];
  }
}

// -------------------------------------------------------- family build --

__global__ void k_bbox(const double* __restrict__ x, int64_t n, double* __restrict__ part,
                       const int32_t* __restrict__ gate) {
  if (*gate == 0) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    for (int c = 0; c < 3; ++c) {
      double v = x[c * n + i];
      lo[c] = fmin(lo[c], v);
      hi[c] = fmax(hi[c], v);
    }
  __shared__ double s[6][256];
  for (int c = 0; c < 3; ++c) { s[c][threadIdx.x] = lo[c]; s[3 + c][threadIdx.x] = hi[c]; }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 3; ++c) {
        s[c][threadIdx.x] = fmin(s[c][threadIdx.x], s[c][threadIdx.x + o]);
        s[3 + c][threadIdx.x] = fmax(s[3 + c][threadIdx.x], s[3 + c][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

// Cells of edge >= delta over the bounding box, doubled until the grid fits
// the allocated cell arrays.  One block reduces the bounding-box partials; a
// non-finite box flags an error and collapses everything into one cell (the
// search stays in bounds).
__global__ __launch_bounds__(256) void k_grid(const double* __restrict__ part, int nb, double delta,
                                              int64_t max_cells, Grid* __restrict__ G,
                                              unsigned long long* __restrict__ ctr, const int32_t* __restrict__ gate) {
  if (*gate == 0) return;
  __shared__ double s[6][256];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nb; b += 256)
    for (int c = 0; c < 3; ++c) {
      v[c] = fmin(v[c], part[6 * b + c]);
      v[3 + c] = fmax(v[3 + c], part[6 * b + 3 + c]);
    }
  for (int c = 0; c < 6; ++c) s[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 3; ++c) {
        s[c][threadIdx.x] = fmin(s[c][threadIdx.x], s[c][threadIdx.x + o]);
        s[3 + c][threadIdx.x] = fmax(s[3 + c][threadIdx.x], s[3 + c][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double lo[3] = {s[0][0], s[1][0], s[2][0]}, hi[3] = {s[3][0], s[4][0], s[5][0]};
  bool ok = true;
  for (int c = 0; c < 3; ++c) ok = ok && isfinite(lo[c]) && isfinite(hi[c]);
  Grid g;
  if (!ok) {
    ctr_add(ctr, C_NONFINITE, 1ull);
    g.lo0 = g.lo1 = g.lo2 = 0.0;
    g.cs = INFINITY;
    g.d0 = g.d1 = g.d2 = 1;
    g.ncell = 1;
    *G = g;
    return;
  }
  double cs = delta * (1.0 + 1e-9);
  int64_t d[3];
  for (;;) {
    double tot = 1.0;
    for (int c = 0; c < 3; ++c) {
      d[c] = (int64_t)floor((hi[c] - lo[c]) / cs) + 1;
      tot *= (double)d[c];
    }
    if (tot <= (double)max_cells) break;
    cs *= 2.0;
  }
  g.lo0 = lo[0]; g.lo1 = lo[1]; g.lo2 = lo[2];
  g.cs = cs;
  g.d0 = d[0]; g.d1 = d[1]; g.d2 = d[2];
  g.ncell = d[0] * d[1] * d[2];
  *G = g;
}

__device__ __forceinline__ int64_t cell_coord(double v, double lo, double cs, int64_t d) {
  double t = floor((v - lo) / cs);
  int64_t k = isfinite(t) ? (int64_t)t : 0;
  return k < 0 ? 0 : (k >= d ? d - 1 : k);
}

__global__ void k_cell_count(const double* __restrict__ x, int64_t n, const Grid* __restrict__ G,
                             int32_t* __restrict__ cellid, int32_t* __restrict__ ccount,
                             const int32_t* __restrict__ gate) {
  if (*gate == 0) return;
  const Grid g = *G;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = cell_coord(x[i], g.lo0, g.cs, g.d0);
    int64_t b = cell_coord(x[n + i], g.lo1, g.cs, g.d1);
    int64_t c = cell_coord(x[2 * n + i], g.lo2, g.cs, g.d2);
    int32_t cid = (int32_t)(a + g.d0 * (b + g.d1 * c));
    cellid[i] = cid;
    atomicAdd(&ccount[cid], 1);
  }
}

__global__ void k_cell_fill(int64_t n, const int32_t* __restrict__ cellid, const int64_t* __restrict__ cstart,
                            int32_t* __restrict__ ccursor, int32_t* __restrict__ cpts,
                            const int32_t* __restrict__ gate) {
  if (*gate == 0) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t cid = cellid[i];
    int32_t pos = atomicAdd(&ccursor[cid], 1);
    cpts[cstart[cid] + pos] = (int32_t)i;
  }
}

// Candidate lists: every point within delta + skin, found with a cell list.
// One wave per point tests the points of the 27 surrounding cells, appends
// hits through a ballot prefix, then places each hit at its rank (ids are
// distinct) so the row comes out ascending.  The three cells along x of a
// (y, z) row are consecutive in cell order, so their points form one
// contiguous range of the cell list: 9 ranges per point.  Runs only when the
// gate is set (first build of a call, or a point moved more than skin/2).
__global__ __launch_bounds__(kWave) void k_family(const double* __restrict__ x, int64_t n, int64_t per,
                                                  const Grid* __restrict__ G, const int32_t* __restrict__ cellid,
                                                  const int64_t* __restrict__ cstart,
                                                  const int32_t* __restrict__ cpts, double d2, int max_f,
                                                  int32_t* __restrict__ ell, int32_t* __restrict__ cnt,
                                                  unsigned long long* __restrict__ ctr,
                                                  const int32_t* __restrict__ gate) {
  extern __shared__ int32_t list[];
  if (*gate == 0) return;
  const int lane = threadIdx.x;
  const Grid g = *G;
  // Grid-stride over points with a capped grid (a multiple of 8, so each
  // block stays on its XCD's contiguous range): cheap to launch when gated off.
  for (int64_t b = blockIdx.x; b < 8 * per; b += gridDim.x) {
    const int64_t i = xcd_point(b, per);
    if (i >= n) continue;
    const double xi = x[i], yi = x[n + i], zi = x[2 * n + i];
    const int64_t cid = cellid[i];
    const int64_t ca = cid % g.d0, cb = (cid / g.d0) % g.d1, cc = cid / (g.d0 * g.d1);
    const int64_t a0 = ca > 0 ? ca - 1 : 0, a1 = ca + 1 < g.d0 ? ca + 1 : g.d0 - 1;
    int count = 0;
    for (int r = 0; r < 9; ++r) {
      const int64_t c3 = cc + (r / 3) - 1, c2 = cb + (r % 3) - 1;
      if (c3 < 0 || c3 >= g.d2 || c2 < 0 || c2 >= g.d1) continue;
      const int64_t crow = g.d0 * (c2 + g.d1 * c3);
      const int64_t s0 = cstart[crow + a0], s1 = cstart[crow + a1 + 1];
      for (int64_t base = s0; base < s1; base += kWave) {
        const int64_t e = base + lane;
        bool hit = false;
        int32_t j = -1;
        if (e < s1) {
          j = cpts[e];
          hit = (j != (int32_t)i) && within(xi, yi, zi, x[j], x[n + j], x[2 * n + j], d2);
        }
        const unsigned long long mask = __ballot(hit);
        const int off = __popcll(mask & ((1ull << lane) - 1ull));
        if (hit && count + off < max_f) list[count + off] = j;
        count += __popcll(mask);
      }
    }
    __syncthreads();
    const int kept = count < max_f ? count : max_f;
    for (int e = lane; e < kept; e += kWave) {
      const int32_t v = list[e];
      int r = 0;
      for (int k = 0; k < kept; ++k) r += list[k] < v;
      ell[i * (int64_t)max_f + r] = v;
    }
    __syncthreads();
    if (lane == 0) {
      cnt[i] = kept;
      if (count > max_f) ctr_add(ctr, C_OVERFLOW, 1ull);
    }
  }
}

// Reverse candidate index: position of i in the (sorted) candidate row of j,
// by binary search; candidates are symmetric, so it exists.  Gated.
__global__ __launch_bounds__(256) void k_cand_rev(int64_t n, int max_c, const int32_t* __restrict__ cand,
                                                  const int32_t* __restrict__ ccnt, int32_t* __restrict__ crev,
                                                  unsigned long long* __restrict__ ctr,
                                                  const int32_t* __restrict__ gate) {
  if (*gate == 0) return;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * max_c;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / max_c;
    const int m = (int)(e - i * max_c);
    if (m >= ccnt[i]) continue;
    const int32_t j = cand[e];
    const int32_t* rj = cand + (int64_t)j * max_c;
    int lo = 0, hi = ccnt[j];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (rj[mid] < (int32_t)i) lo = mid + 1; else hi = mid;
    }
    const bool found = lo < ccnt[j] && rj[lo] == (int32_t)i;
    crev[e] = found ? lo : -1;
    if (!found) ctr_add(ctr, C_OVERFLOW, 1ull);
  }
}

__global__ void k_save_ref(const double* __restrict__ x, double* __restrict__ xref, int64_t m,
                           unsigned long long* __restrict__ ctr, const int32_t* __restrict__ gate) {
  if (*gate == 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr_add(ctr, C_REBUILD, 1ull);   // one candidate rebuild
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
    xref[e] = x[e];
}

// Sets the gate when some point moved more than skin/2 since the candidate
// lists were built: then a pair within delta now was within delta + skin then.
__global__ void k_check_skin(const double* __restrict__ x, const double* __restrict__ xref, int64_t n,
                             double lim2, int32_t* __restrict__ gate) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double a = x[i] - xref[i], b = x[n + i] - xref[n + i], c = x[2 * n + i] - xref[2 * n + i];
    const double d = a * a + b * b + c * c;
    if (!(d <= lim2)) *gate = 1;
  }
}

// Family of every point in the current configuration (Eq. 1): a group of
// lanes per point filters its candidate row with the exact predicate; the
// ballot bits, kept per candidate slot, give each member its slot in the row
// (the members before it), so rows stay ascending.  LPP: lanes per point, a
// whole wave, half a wave, or one 16-lane row (four points per wave, for
// candidate lists of a few dozen).
template <int LPP>
__global__ __launch_bounds__(256) void k_filter(const double* __restrict__ xv, int64_t n, int max_c, int max_f,
                                                const int32_t* __restrict__ cand, const int32_t* __restrict__ ccnt,
                                                double d2, unsigned long long* __restrict__ fbits,
                                                int32_t* __restrict__ cnt, unsigned long long* __restrict__ ctr) {
  static_assert(LPP == kWave || LPP == 32 || LPP == 16, "a point per wave or per 32- or 16-lane group");
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (LPP - 1), sh = lane & ~(LPP - 1);     // lane in the group, the group's first bit
  const unsigned long long gmask = LPP == kWave ? ~0ull : ((1ull << LPP) - 1ull) << sh;
  const XcdWalk W = xcd_walk_groups(n, 256 / LPP, threadIdx.x / LPP);
  int wmax = 0;
  const double4* P4 = reinterpret_cast<const double4*>(xv);     // packed records: x, y, z, V first
  for (int64_t i = W.first; i < W.end; i += W.stride) {
    const double4 pi = P4[2 * i];
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    const int nc = ccnt[i];
    int count = 0;
    for (int base = 0; base < nc; base += LPP) {
      const int c = base + sub;
      bool hit = false;
      if (c < nc) {
        const int32_t j = cand[i * (int64_t)max_c + c];
        const double4 pj = P4[2 * (int64_t)j];                     // one 32-byte read per candidate
        hit = within(xi, yi, zi, pj.x, pj.y, pj.z, d2);
      }
      const unsigned long long mask = __ballot(hit) & gmask;     // this group's hits
      // membership bit of each candidate slot, 64 slots to a word (slots
      // past the count read as clear)
      if constexpr (LPP == kWave) {
        if (lane == 0) fbits[i * (int64_t)(max_c / 64) + base / 64] = mask;
      } else if constexpr (LPP == 32) {
        if (sub == 0)
          reinterpret_cast<uint32_t*>(fbits)[i * (int64_t)(max_c / 32) + base / 32] = (uint32_t)(mask >> sh);
      } else {
        if (sub == 0)
          reinterpret_cast<uint16_t*>(fbits)[i * (int64_t)(max_c / 16) + base / 16] = (uint16_t)(mask >> sh);
      }
      count += __popcll(mask);
    }
    if (sub == 0) {
      cnt[i] = count < max_f ? count : max_f;
      if (count > max_f) ctr_add(ctr, C_OVERFLOW, 1ull);
    }
    wmax = wmax > count ? wmax : count;
  }
  wmax = wave_max_i(wmax);
  if (lane == 0 && wmax > 0) ctr_max(ctr, C_MAXFAM, (unsigned long long)wmax);
}

// Position in its point's family row of the member in candidate slot c (the
// members in the slots before it), or -1 if the slot holds no member; b are
// the point's membership words.
__device__ __forceinline__ int member_pos(const unsigned long long* __restrict__ b, int c) {
  const unsigned long long w = b[c >> 6];
  if (!((w >> (c & 63)) & 1ull)) return -1;
  int p = __popcll(w & ((1ull << (c & 63)) - 1ull));
  for (int k = 0; k < (c >> 6); ++k) p += __popcll(b[k]);
  return p;
}

// A group of LPP lanes per point over its candidate slots: for every member, the
// CSR column and the reverse-bond slot rev[(i,j)] = slot of (j,i), found
// through the reverse candidate index (no search) and the membership words
// of j (a few bytes per point, which stay in L2, where a table of positions
// per candidate slot would not).
template <int LPP>
__global__ __launch_bounds__(256) void k_compact(int64_t n, int max_c, int max_f, const int32_t* __restrict__ cand,
                                                 const int32_t* __restrict__ ccnt, const int32_t* __restrict__ crev,
                                                 const unsigned long long* __restrict__ fbits,
                                                 const int64_t* __restrict__ row, int32_t* __restrict__ col,
                                                 int32_t* __restrict__ rev, unsigned long long* __restrict__ ctr) {
  const int sub = threadIdx.x & (LPP - 1);
  const int nw = max_c / 64;
  const XcdWalk W = xcd_walk_groups(n, 256 / LPP, threadIdx.x / LPP);
  for (int64_t i = W.first; i < W.end; i += W.stride) {
    const int nc = ccnt[i];
    const int64_t r0 = row[i];
    const int64_t e0 = i * (int64_t)max_c;
    const unsigned long long* bi = fbits + i * nw;
    for (int c = sub; c < nc; c += LPP) {
      const int pm = member_pos(bi, c);
      if (pm < 0 || pm >= max_f) continue;
      const int64_t s = r0 + pm;
      const int32_t j = cand[e0 + c];
      col[s] = j;
      const int cr = crev[e0 + c];
      const int pr = cr >= 0 ? member_pos(fbits + (int64_t)j * nw, cr) : -1;
      // The exact predicate is symmetric, so (j,i) is a member of row j.
      const bool ok = pr >= 0 && pr < max_f;
      rev[s] = (int32_t)(ok ? row[j] + pr : s);
      if (!ok) ctr_add(ctr, C_OVERFLOW, 1ull);
    }
  }
}

// ----------------------------------------------------- constitutive model --

// Apparent pre-consolidation P(p_c) = -exp(b1) (-p_c)^b2 (Eq. 45) and its
// slope dP/dp_c (Eq. 89).  With b1 = 0 and b2 = 1 they are p_c and 1, taken
// without the transcendental calls (the Newton iterations of the plastic
// bonds evaluate both every iteration).  LinP = true compiles that case
// alone: such code carries none of the registers of the general power (the
// bond kernels' return map is their register peak).
template <bool LinP = false>
__host__ __device__ __forceinline__ double apparent_pc(const DevParams& P, double pc) {
  if (LinP || (P.b1 == 0.0 && P.b2 == 1.0)) return pc;
  return -exp(P.b1) * pow(-pc, P.b2);               // Eq. 45
}
template <bool LinP = false>
__host__ __device__ __forceinline__ double apparent_pc_slope(const DevParams& P, double pc) {
  if (LinP || (P.b1 == 0.0 && P.b2 == 1.0)) return 1.0;
  return P.b2 * exp(P.b1) * pow(-pc, P.b2 - 1.0);   // Eq. 89
}

__host__ __device__ __forceinline__ double yield_f(const DevParams& P, double p, double q, double pcb) {
  return q * q * P.iM2 + p * (p - pcb);             // Eq. 40
}

// Retention curve, Eq. 15 read with exponent -(n-1)/n, suction in kPa, void
// ratio e = phi/(1-phi).
__host__ __device__ double swrc(const DevParams& P, double J, double phi, double s) {
  if (!(s > 0.0)) return 1.0;
  const double e = phi / (1.0 - phi);
  const double arg = P.a1 * pow(e, P.a2) * J * (s * 1e-3);
  return pow(1.0 + pow(arg, P.n_vg), -(P.n_vg - 1.0) / P.n_vg);
}

// Where Newton stalls, the same backward-Euler equations are solved through
// the consistency parameter g = c f >= 0.  With it q = q_tr/(1 + 6 mu g/M^2),
// p = (p_tr + K g P)/(1 + 2 K g) (hence 2p - P = (2 p_tr - P)/(1 + 2 K g)) and
// p_c solves p_c = p_c,n exp(-g (2 p_tr - P(p_c)) / ((lam - kap)(1 + 2 K g))),
// a strictly increasing equation in p_c; g itself is the root of
// g - c f(p, q, P) on [0, inf), where it changes sign once.
template <bool LinP>
struct ConsistencySolve {
  double K, mu, M2, lk, b1, b2, c, ptr, qtr, pcn;
  __host__ __device__ double Pb(double pc) const {
    return LinP || (b1 == 0.0 && b2 == 1.0) ? pc : -exp(b1) * pow(-pc, b2);
  }
  __host__ __device__ double dPb(double pc) const {
    return LinP || (b1 == 0.0 && b2 == 1.0) ? 1.0 : b2 * exp(b1) * pow(-pc, b2 - 1.0);
  }
  __host__ __device__ double pc_for(double g) const {
    const double A = g / (lk * (1.0 + 2.0 * K * g));
    double hi = 0.0, lo = pcn;
    for (int k = 0; k < 4000; ++k) {             // bracket: h(lo) <= 0 < h(0-)
      if (lo - pcn * exp(-A * (2.0 * ptr - Pb(lo))) <= 0.0) break;
      hi = lo;
      lo *= 2.0;
    }
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
      const double E = exp(-A * (2.0 * ptr - Pb(x)));
      const double h = x - pcn * E;
      if (h > 0.0) hi = x; else lo = x;
      const double dh = 1.0 - pcn * E * A * dPb(x);
      double xn = x - h / dh;
      if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
      const bool done = fabs(xn - x) <= 1e-16 * fabs(x);
      x = xn;
      if (done || hi - lo <= 1e-16 * fabs(lo)) break;
    }
    return x;
  }
  __host__ __device__ void at(double g, double* x) const {
    x[2] = pc_for(g);
    x[0] = (ptr + K * g * Pb(x[2])) / (1.0 + 2.0 * K * g);
    x[1] = qtr / (1.0 + 6.0 * mu * g / M2);
  }
  __host__ __device__ double resid(double g) const {
    double x[3];
    at(g, x);
    return g - c * (x[1] * x[1] / M2 + x[0] * (x[0] - Pb(x[2])));
  }
  __host__ __device__ void solve(double ftr, double* x) const {
    double lo = 0.0, hi = c * ftr, rlo = -c * ftr, rhi = resid(hi);
    for (int k = 0; k < 2000 && rhi < 0.0; ++k) { lo = hi; rlo = rhi; hi *= 2.0; rhi = resid(hi); }
    for (int it = 0; it < 400 && hi - lo > 2e-16 * hi; ++it) {
      // secant inside the bracket once it is narrow, bisection before
      double g = (hi - lo > 1e-3 * hi) ? 0.5 * (lo + hi) : lo - rlo * (hi - lo) / (rhi - rlo);
      if (!(g > lo && g < hi)) g = 0.5 * (lo + hi);
      const double r = resid(g);
      if (r == 0.0) { lo = hi = g; break; }
      if (r > 0.0) { hi = g; rhi = r; } else { lo = g; rlo = r; }
    }
    at(0.5 * (lo + hi), x);
  }
};

// Backward-Euler Perzyna update in the invariants (Eqs. 70-76): residuals
// r1 = p - p_tr + K c f f_p, r2 = q - q_tr + 3 mu c f f_q,
// r3 = p_c - p_c,n exp(-c f f_p / (lam - kap)) with c = dt/eta, solved by
// Newton with the exact tangent; steps are halved to stay in
// {f > 0, q >= 0, p_c < 0}, where the solution lies.  Returns the iteration
// count (0 elastic) or -1.
// Pn: the apparent pre-consolidation of pcn (Eq. 45), the same for every
// bond of a point.
template <bool LinP = false>
__host__ __device__ int return_map_pn(const DevParams& P, double dt, const double* sn, double pcn, double Pn,
                                      const double* de, double* so, double* pco) {
  constexpr double kThird = 1.0 / 3.0;
  const double tr = de[0] + de[1] + de[2];
  double st[6];
#pragma unroll
  for (int k = 0; k < 6; ++k)
    st[k] = sn[k] + (k < 3 ? P.K * tr : 0.0) + 2.0 * P.mu * (de[k] - (k < 3 ? tr * kThird : 0.0));
  const double ptr = (st[0] + st[1] + st[2]) * kThird;
  double s[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = st[k] - (k < 3 ? ptr : 0.0);
  const double qtr = sqrt(1.5 * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2] +
                                 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5])));
  if (__builtin_expect(!(yield_f(P, ptr, qtr, Pn) > 0.0), 1)) {   // elastic: the common case, laid out first
#pragma unroll
    for (int k = 0; k < 6; ++k) so[k] = st[k];
    *pco = pcn;
    return 0;
  }
  const double c = dt / P.eta, M2 = P.M * P.M, lk = P.lam - P.kap;
  const double sref = fmax(fabs(ptr), fmax(qtr, fabs(Pn)));
  const double pref = fabs(pcn);
  double p = ptr, q = qtr, pc = pcn;
  int it = 0;
  bool conv = false, stalled = false;
  for (;;) {
    const double Pb = apparent_pc<LinP>(P, pc);
    const double dP = apparent_pc_slope<LinP>(P, pc);            // Eq. 89
    const double f = yield_f(P, p, q, Pb);
    const double fp = 2.0 * p - Pb, fq = 2.0 * q / M2, fc = -p * dP;
    const double E = exp(-c * f * fp / lk);
    const double r1 = p - ptr + P.K * c * f * fp;
    const double r2 = q - qtr + 3.0 * P.mu * c * f * fq;
    const double r3 = pc - pcn * E;
    if (fabs(r1) <= P.newton_tol * sref && fabs(r2) <= P.newton_tol * sref && fabs(r3) <= P.newton_tol * pref) {
      conv = true;
      break;
    }
    if (__builtin_expect(it >= P.newton_maxit || stalled, 0)) {
      ConsistencySolve<LinP> B{P.K, P.mu, M2, lk, P.b1, P.b2, c, ptr, qtr, pcn};
      double xb[3];
      B.solve(yield_f(P, ptr, qtr, Pn), xb);
      p = xb[0];
      q = xb[1];
      pc = xb[2];
      const double Pb2 = apparent_pc<LinP>(P, pc);
      const double f2 = yield_f(P, p, q, Pb2), fp2 = 2.0 * p - Pb2;
      const double e1 = p - ptr + P.K * c * f2 * fp2;
      const double e2 = q - qtr + 3.0 * P.mu * c * f2 * 2.0 * q / M2;
      const double e3 = pc - pcn * exp(-c * f2 * fp2 / lk);
      conv = fabs(e1) <= 1e3 * P.newton_tol * sref && fabs(e2) <= 1e3 * P.newton_tol * sref &&
             fabs(e3) <= 1e3 * P.newton_tol * pref;
      it = P.newton_maxit + 1;
      break;
    }
    // d(f fp)/dx and d(f fq)/dx
    const double gp = fp * fp + 2.0 * f, gq = fq * fp, gc = fc * fp - f * dP;
    const double hp = fp * fq, hq = fq * fq + f * 2.0 / M2, hc = fc * fq;
    const double k1 = P.K * c, k2 = 3.0 * P.mu * c, k3 = pcn * E * c / lk;
    const double a11 = 1.0 + k1 * gp, a12 = k1 * gq, a13 = k1 * gc;
    const double a21 = k2 * hp, a22 = 1.0 + k2 * hq, a23 = k2 * hc;
    const double a31 = k3 * gp, a32 = k3 * gq, a33 = 1.0 + k3 * gc;
    // Cramer's rule for A dx = -r
    const double c11 = a22 * a33 - a23 * a32, c12 = a23 * a31 - a21 * a33, c13 = a21 * a32 - a22 * a31;
    const double det = a11 * c11 + a12 * c12 + a13 * c13;
    const double b1 = -r1, b2 = -r2, b3 = -r3;
    const double dx1 = (b1 * c11 + a12 * (a23 * b3 - b2 * a33) + a13 * (b2 * a32 - a22 * b3)) / det;
    const double dx2 = (a11 * (b2 * a33 - a23 * b3) + b1 * c12 + a13 * (a21 * b3 - b2 * a31)) / det;
    const double dx3 = (a11 * (a22 * b3 - b2 * a32) + a12 * (b2 * a31 - a21 * b3) + b1 * c13) / det;
    double stp = 1.0;
    for (int h = 0; h < 60; ++h) {
      const double pt = p + stp * dx1, qt = q + stp * dx2, ct = pc + stp * dx3;
      if (ct < 0.0 && qt >= 0.0 && yield_f(P, pt, qt, apparent_pc<LinP>(P, ct)) > 0.0) break;
      stp *= 0.5;
    }
    p += stp * dx1;
    q += stp * dx2;
    pc += stp * dx3;
    ++it;
    stalled = stp < 1e-6;
  }
  const double ratio = qtr > 0.0 ? q / qtr : 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) so[k] = (k < 3 ? p : 0.0) + ratio * s[k];
  *pco = pc;
  if (!conv) return -1;
  return it > 0 ? it : 1;
}

__host__ __device__ int return_map(const DevParams& P, double dt, const double* sn, double pcn, const double* de,
                                   double* so, double* pco) {
  return return_map_pn(P, dt, sn, pcn, apparent_pc(P, pcn), de, so, pco);
}

__host__ __device__ __forceinline__ double det3s(double a, double b, double c, double d, double e, double f) {
  // symmetric [[a f e],[f b d],[e d c]]
  return a * (b * c - d * d) - f * (f * c - d * e) + e * (f * d - b * e);
}

// ------------------------------------------------ per-bond tail and its reverse --
// The per-bond tail of the step, as a function of the sub-horizon sums:
//   K_ij^{-1}; L = N K^{-1}; de = dt sym(L) (Eqs. 25-26, 59); the Perzyna
//   return map (Section 3.2.1); Q = sigma_ij + S_r s 1 (Eq. 32, p_w = -s);
//   M_j = w_j Q K^{-1}, the factor of the conjugate force states.
// tail_reverse is its hand-written adjoint, with the elastic/plastic branch
// frozen; the return map is differentiated through the implicit-function
// theorem at the converged point.  Both run on the device and on the host
// (for the host self-check against finite differences).

struct TailFwd {
  double Ki[6];      // K^{-1}, Voigt
  double de[6];      // strain increment, Voigt (tensor shears)
  double sg[6];      // bond stress after the update
  double pc;         // bond p_c after the update
  double M[9];       // w Q K^{-1}, row-major
  int branch;        // 0 elastic, > 0 plastic (Newton iterations), < 0 no convergence
};

// Inverse of a symmetric 3x3 in Voigt order (xx, yy, zz, yz, xz, xy).
__host__ __device__ __forceinline__ double sym_inverse(const double* K, double* Ki) {
  const double a = K[0], b = K[1], c = K[2], d = K[3], e = K[4], f = K[5];
  const double det = det3s(a, b, c, d, e, f);
  Ki[0] = (b * c - d * d) / det;
  Ki[1] = (a * c - e * e) / det;
  Ki[2] = (a * b - f * f) / det;
  Ki[3] = (e * f - a * d) / det;
  Ki[4] = (f * d - b * e) / det;
  Ki[5] = (d * e - f * c) / det;
  return det;
}

// Whether a shape tensor (Voigt xx, yy, zz, yz, xz, xy) summed over `count`
// members can be inverted: not when it is degenerate, with fewer members than
// dimensions or det K <= 1e-12 (tr K / d)^d.  In plane strain (x-z plane)
// only the x-z block is inverted and the y row and column of the inverse are
// zero; shape_inverse tests and inverts.
__host__ __device__ __forceinline__ bool shape_regular(bool plane, const double* K, int count) {
  if (!plane) {
    const double dK = det3s(K[0], K[1], K[2], K[3], K[4], K[5]);
    const double tk = (K[0] + K[1] + K[2]) / 3.0;
    return count >= 3 && dK > 1e-12 * tk * tk * tk;
  }
  const double d2 = K[0] * K[2] - K[4] * K[4];
  const double tr = (K[0] + K[2]) / 2.0;
  return count >= 2 && d2 > 1e-12 * tr * tr;
}

// The inverse itself, for a tensor shape_regular accepts.
__host__ __device__ __forceinline__ void shape_inverse_of(bool plane, const double* K, double* Ki) {
  if (!plane) {
    sym_inverse(K, Ki);
    return;
  }
  const double a = K[0], c = K[2], e = K[4];
  const double id = 1.0 / (a * c - e * e);
  Ki[0] = c * id; Ki[1] = 0.0; Ki[2] = a * id; Ki[3] = 0.0; Ki[4] = -e * id; Ki[5] = 0.0;
}

__host__ __device__ __forceinline__ bool shape_inverse(bool plane, const double* K, int count, double* Ki) {
  if (!shape_regular(plane, K, count)) return false;
  shape_inverse_of(plane, K, Ki);
  return true;
}

__host__ __device__ __forceinline__ void sym_full(const double* v, double* A) {
  A[0] = v[0]; A[1] = v[5]; A[2] = v[4];
  A[3] = v[5]; A[4] = v[1]; A[5] = v[3];
  A[6] = v[4]; A[7] = v[3]; A[8] = v[2];
}

__host__ __device__ __forceinline__ void mat3_mul(const double* A, const double* B, double* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

// Gradient with respect to the six unique entries of a symmetric matrix,
// from the gradient G with respect to its nine entries.
__host__ __device__ __forceinline__ void unique_grad(const double* G, double* g) {
  g[0] = G[0]; g[1] = G[4]; g[2] = G[8];
  g[3] = G[5] + G[7]; g[4] = G[2] + G[6]; g[5] = G[1] + G[3];
}

// K^{-1} and the strain increment dt sym(N K^{-1}) of a bond (Eqs. 25-26, 59).
__host__ __device__ __forceinline__ void tail_kinematics(bool plane, const double* K, const double* N, double dt,
                                                         TailFwd& F) {
  shape_inverse_of(plane, K, F.Ki);
  double KiF[9], L[9];
  sym_full(F.Ki, KiF);
  mat3_mul(N, KiF, L);
  F.de[0] = dt * L[0]; F.de[1] = dt * L[4]; F.de[2] = dt * L[8];
  F.de[3] = dt * 0.5 * (L[5] + L[7]); F.de[4] = dt * 0.5 * (L[2] + L[6]); F.de[5] = dt * 0.5 * (L[1] + L[3]);
}

// Pn: apparent pre-consolidation of pc (Eq. 45).
template <bool LinP = false>
__host__ __device__ void tail_forward_pn(const DevParams& P, const double* K, const double* N, const double* sig,
                                         double pc, double Pn, double Srs, double w, double dt, TailFwd& F) {
  tail_kinematics(P.plane != 0, K, N, dt, F);
  double KiF[9];
  sym_full(F.Ki, KiF);
  if (dt == 0.0) {
    for (int k = 0; k < 6; ++k) F.sg[k] = sig[k];
    F.pc = pc;
    F.branch = 0;
  } else {
    F.branch = return_map_pn<LinP>(P, dt, sig, pc, Pn, F.de, F.sg, &F.pc);
  }
  double Q[6] = {F.sg[0] + Srs, F.sg[1] + Srs, F.sg[2] + Srs, F.sg[3], F.sg[4], F.sg[5]};
  double QF[9], SK[9];
  sym_full(Q, QF);
  mat3_mul(QF, KiF, SK);
  for (int k = 0; k < 9; ++k) F.M[k] = w * SK[k];
}

__host__ __device__ void tail_forward(const DevParams& P, const double* K, const double* N, const double* sig,
                                      double pc, double Srs, double w, double dt, TailFwd& F) {
  tail_forward_pn(P, K, N, sig, pc, apparent_pc(P, pc), Srs, w, dt, F);
}

// Adjoint of the return map at fixed branch: given the adjoints of the
// updated bond stress (sgb, Voigt components) and p_c, accumulate those of
// the point stress, p_c,n, the strain increment and (M, lam, kap, eta).
template <bool LinP = false>
__host__ __device__ void rm_reverse(const DevParams& P, double dt, const double* sn, double pcn, const double* de,
                                    const double* so, double pco, int branch, const double* sgb, double pcb,
                                    double* snb, double* pcnb, double* deb, double* thb) {
  constexpr double kThird = 1.0 / 3.0;             // as the forward trial state
  const double tr = de[0] + de[1] + de[2];
  double st[6], s[6];
  for (int k = 0; k < 6; ++k)
    st[k] = sn[k] + (k < 3 ? P.K * tr : 0.0) + 2.0 * P.mu * (de[k] - (k < 3 ? tr * kThird : 0.0));
  const double ptr = (st[0] + st[1] + st[2]) * kThird;
  for (int k = 0; k < 6; ++k) s[k] = st[k] - (k < 3 ? ptr : 0.0);
  const double qtr = sqrt(1.5 * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5])));
  double stb[6];
  if (__builtin_expect(branch == 0, 1)) {          // elastic: the common case, laid out first
    for (int k = 0; k < 6; ++k) stb[k] = sgb[k];
    *pcnb += pcb;
  } else {
    const double p = (so[0] + so[1] + so[2]) / 3.0;
    const double d0 = so[0] - p, d1 = so[1] - p, d2 = so[2] - p;
    const double q = sqrt(1.5 * (d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * (so[3] * so[3] + so[4] * so[4] + so[5] * so[5])));
    const double ratio = qtr > 0.0 ? q / qtr : 0.0;
    // sigma = p 1 + ratio s_tr
    const double pbar = sgb[0] + sgb[1] + sgb[2];
    double ratiob = 0.0, sb[6];
    for (int k = 0; k < 6; ++k) {
      ratiob += sgb[k] * s[k];
      sb[k] = ratio * sgb[k];
    }
    const double qbar = qtr > 0.0 ? ratiob / qtr : 0.0;
    double qtrb = qtr > 0.0 ? -ratiob * q / (qtr * qtr) : 0.0;
    // implicit function theorem at the solution x = (p, q, pc)
    const double c = dt / P.eta, M2 = P.M * P.M, lk = P.lam - P.kap;
    const double Pb = apparent_pc<LinP>(P, pco);
    const double dP = apparent_pc_slope<LinP>(P, pco);
    const double f = yield_f(P, p, q, Pb);
    const double fp = 2.0 * p - Pb, fq = 2.0 * q / M2, fc = -p * dP;
    const double E = exp(-c * f * fp / lk);
    const double gp = fp * fp + 2.0 * f, gq = fq * fp, gc = fc * fp - f * dP;
    const double hp = fp * fq, hq = fq * fq + f * 2.0 / M2, hc = fc * fq;
    const double k1 = P.K * c, k2 = 3.0 * P.mu * c, k3 = pcn * E * c / lk;
    const double A[9] = {1.0 + k1 * gp, k1 * gq, k1 * gc, k2 * hp, 1.0 + k2 * hq, k2 * hc,
                         k3 * gp, k3 * gq, 1.0 + k3 * gc};
    // mu = A^{-T} xbar by Cramer's rule on A^T
    const double T[9] = {A[0], A[3], A[6], A[1], A[4], A[7], A[2], A[5], A[8]};
    const double xb[3] = {pbar, qbar, pcb};
    const double c11 = T[4] * T[8] - T[5] * T[7], c12 = T[5] * T[6] - T[3] * T[8], c13 = T[3] * T[7] - T[4] * T[6];
    const double det = T[0] * c11 + T[1] * c12 + T[2] * c13;
    const double m0 = (xb[0] * c11 + T[1] * (T[5] * xb[2] - xb[1] * T[8]) + T[2] * (xb[1] * T[7] - T[4] * xb[2])) / det;
    const double m1 = (T[0] * (xb[1] * T[8] - T[5] * xb[2]) + xb[0] * c12 + T[2] * (T[3] * xb[2] - xb[1] * T[6])) / det;
    const double m2 = (T[0] * (T[4] * xb[2] - xb[1] * T[7]) + T[1] * (xb[1] * T[6] - T[3] * xb[2]) + xb[0] * c13) / det;
    // r1 = p - ptr + K c f fp, r2 = q - qtr + 3 mu c f fq, r3 = pc - pcn E
    const double ptrb = m0;
    qtrb += m1;
    *pcnb += m2 * E;
    // parameters: M (slope), lam, kap, eta
    const double dfM = -2.0 * q * q / (M2 * P.M), dhM = -4.0 * q / (M2 * P.M);
    const double r1M = k1 * dfM * fp, r2M = k2 * (dfM * fq + f * dhM), r3M = pcn * E * c * fp * dfM / lk;
    const double r3lk = -pcn * E * c * f * fp / (lk * lk);
    const double dcdeta = -c / P.eta;
    const double r1e = P.K * f * fp * dcdeta, r2e = 3.0 * P.mu * f * fq * dcdeta, r3e = pcn * E * f * fp / lk * dcdeta;
    thb[0] -= m0 * r1M + m1 * r2M + m2 * r3M;
    thb[1] -= m2 * r3lk;
    thb[2] += m2 * r3lk;
    thb[3] -= m0 * r1e + m1 * r2e + m2 * r3e;
    // trial state: p_tr, s_tr, q_tr from st
    if (qtr > 0.0) {
      const double wgt[6] = {1, 1, 1, 2, 2, 2};
      for (int k = 0; k < 6; ++k) sb[k] += qtrb * 1.5 * wgt[k] * s[k] / qtr;
    }
    const double ssum = sb[0] + sb[1] + sb[2];
    for (int k = 0; k < 6; ++k) stb[k] = sb[k] + (k < 3 ? (ptrb - ssum) / 3.0 : 0.0);
  }
  // sigma_tr = sigma_n + K tr 1 + 2 mu dev(de)
  const double stsum = stb[0] + stb[1] + stb[2];
  for (int k = 0; k < 6; ++k) {
    snb[k] += stb[k];
    deb[k] += 2.0 * P.mu * stb[k] + (k < 3 ? P.K * stsum - 2.0 * P.mu * stsum / 3.0 : 0.0);
  }
}

// Adjoint of tail_forward: from the adjoints of M (9) and of the bond state
// (sgb_ext, pcb_ext, e.g. from the history average) to those of K (unique
// entries), N (9), the point stress and p_c, S_r s, w and the parameters.
template <bool LinP = false>
__host__ __device__ void tail_reverse(const DevParams& P, const double* K, const double* N, const double* sig,
                                      double pc, double Srs, double w, double dt, const TailFwd& F,
                                      const double* Mb, const double* sgb_ext, double pcb_ext, double* Kb,
                                      double* Nb, double* sigb, double* pcbp, double* Srsb, double* wb,
                                      double* thb) {
  double KiF[9], QF[9], SK[9];
  sym_full(F.Ki, KiF);
  const double Q[6] = {F.sg[0] + Srs, F.sg[1] + Srs, F.sg[2] + Srs, F.sg[3], F.sg[4], F.sg[5]};
  sym_full(Q, QF);
  mat3_mul(QF, KiF, SK);
  double SKb[9];
  double wbar = 0.0;
  for (int k = 0; k < 9; ++k) {
    SKb[k] = w * Mb[k];
    wbar += Mb[k] * SK[k];
  }
  *wb += wbar;
  // SK = Q Ki: Qbar = SKb Ki^T, Kibar = Q^T SKb (both matrices symmetric)
  double QbF[9], KibF[9];
  mat3_mul(SKb, KiF, QbF);
  mat3_mul(QF, SKb, KibF);
  double Qb[6];
  unique_grad(QbF, Qb);
  *Srsb += Qb[0] + Qb[1] + Qb[2];
  double sgb[6];
  for (int k = 0; k < 6; ++k) sgb[k] = Qb[k] + sgb_ext[k];
  double deb[6] = {0, 0, 0, 0, 0, 0};
  if (dt == 0.0) {
    for (int k = 0; k < 6; ++k) sigb[k] += sgb[k];
    *pcbp += pcb_ext;
  } else {
    rm_reverse<LinP>(P, dt, sig, pc, F.de, F.sg, F.pc, F.branch, sgb, pcb_ext, sigb, pcbp, deb, thb);
  }
  // de = dt sym(L): Lbar
  double Lb[9] = {dt * deb[0], 0.5 * dt * deb[5], 0.5 * dt * deb[4],
                  0.5 * dt * deb[5], dt * deb[1], 0.5 * dt * deb[3],
                  0.5 * dt * deb[4], 0.5 * dt * deb[3], dt * deb[2]};
  // L = N Ki: Nbar = Lb Ki^T, Kibar += N^T Lb
  mat3_mul(Lb, KiF, Nb);
  double NT[9] = {N[0], N[3], N[6], N[1], N[4], N[7], N[2], N[5], N[8]};
  double t[9];
  mat3_mul(NT, Lb, t);
  for (int k = 0; k < 9; ++k) KibF[k] += t[k];
  // Ki = K^{-1}: Kbar = -Ki Kibar Ki
  double u[9], KbF[9];
  mat3_mul(KiF, KibF, u);
  mat3_mul(u, KiF, KbF);
  for (int k = 0; k < 9; ++k) KbF[k] = -KbF[k];
  unique_grad(KbF, Kb);
}

// ---------------------------------------------------------- bond kernel --

enum { MODE_STEP = 0, MODE_FORCES = 1 };

struct BondArgs {
  int64_t n, per;
  const int64_t* row;
  const int32_t* col;
  const double* x;        // 3n current positions
  const double* vh;       // 3n velocities used for relative velocities
  const double* vol_n;    // V^n, quadrature weights of this step
  const double* J;
  const double* phi;
  const double* s;
  const double* sig[6];   // point history in
  const double* pc;
  // point outputs (state arrays in step mode, scratch otherwise)
  double* J_out;
  double* vol_out;
  double* phi_out;
  double* Sr_out;
  double* mass_out;
  double* sig_out[6];
  double* pc_out;
  void* T;                // bond force states, CSR order, one (x, y, z, 0) record per bond
                          // (double, or float in mixed precision); V_i T_ik where fown is set
  double* pk;             // 2n: apparent pre-consolidation of p_c,i and 1/V_H,i (point kinematics)
  const double* xv;       // 8n: x (3), V^n, v_half (3), 0 per point
  double* hist;           // history on the bonds: 8 per bond (sigma, p_c, 0), written; or null
  const double* hist_old; // the bond states of the previous step (8 per bond)
  const int64_t* hmap;    // per bond: its slot in hist_old, or -1 (a new bond starts from its point)
  double* fown;           // 3n: sum_k T_ik V_k of each point's own force states (FP64); or null
  double dt_inc;
  int max_f;
  unsigned long long* ctr;
};

// LDS records of one family member, 16-byte aligned so that each is read
// with ds_read_b128 (the adjoint's bond kernel): positions, zeta_ik with V_k,
// ydot_ik; the sub-horizon force-state factors are 9 values per bond, padded
// to a 16-byte multiple.
template <class T>
struct alignas(16) Quad {
  T v[4];
};
template <class Acc>
struct alignas(16) MRec {
  Acc v[sizeof(Acc) == 8 ? 10 : 12];
};

// ------------------------------------------------------ point kinematics --
// One 64-byte record per point for the bond pass's gathers of neighbour
// data: x (3), V^n, v_half (3), 0.
__global__ void k_pack(int64_t n, const double* __restrict__ x, const double* __restrict__ vh,
                       const double* __restrict__ vol_n, double* __restrict__ xv) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double4* r = reinterpret_cast<double4*>(xv + 8 * i);
    r[0] = make_double4(x[i], x[n + i], x[2 * n + i], vol_n[i]);
    r[1] = make_double4(vh[i], vh[n + i], vh[2 * n + i], 0.0);
  }
}

// Point kinematics of the step (Eqs. 5, 8, 15-17, 48), one wave per point:
// the full-horizon shape tensor K_i, velocity-gradient sum N_i and family
// volume V_H in FP64, then lane 0 updates J, V, phi, S_r and the mass and
// stores the apparent pre-consolidation of p_c,i (Eq. 45) and 1/V_H, which
// every bond of i uses.  With geometry at n+1 the step's deformation
// increment F_D satisfies F_D^{-1} = I - dt L_i (Eq. 17 in updated
// Lagrangian form).
//
// In the standard correspondence mode (Eq. 14) the same wave also updates
// the point's stress from L_i by the return map and writes the force states
// T_ik = (sigma_i + S_r s 1) K_i^{-1} zeta_ik of all its bonds; the bond
// kernel does not run.  TS: storage type of the force states.
// Point update from the full-horizon sums K_i, N_i and V_H,i: volume ratio
// of the step from L_i (Eqs. 16-17), porosity, saturation (Eq. 15), mass
// (Eq. 48), and the per-point factors the bond kernel reads (apparent
// pre-consolidation of p_c,i, Eq. 45, and 1/V_H,i).
__device__ __forceinline__ void point_update(const BondArgs& A, const DevParams& P, int64_t i, int nf,
                                             const double* Kp, const double* Np, double Vp) {
  const int64_t n = A.n;
  double Jd = 1.0;
  double Ki[6];
  if (shape_inverse(P.plane != 0, Kp, nf, Ki)) {
    const double Ki9[9] = {Ki[0], Ki[5], Ki[4], Ki[5], Ki[1], Ki[3], Ki[4], Ki[3], Ki[2]};
    double B[9];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) {
        const double L = Np[3 * r] * Ki9[cc] + Np[3 * r + 1] * Ki9[3 + cc] + Np[3 * r + 2] * Ki9[6 + cc];
        B[3 * r + cc] = (r == cc ? 1.0 : 0.0) - A.dt_inc * L;
      }
    const double dB = B[0] * (B[4] * B[8] - B[5] * B[7]) - B[1] * (B[3] * B[8] - B[5] * B[6]) +
                      B[2] * (B[3] * B[7] - B[4] * B[6]);
    Jd = 1.0 / dB;
  }
  const double Jn = A.J[i] * Jd;
  const double Vn = A.vol_n[i] * Jd;
  const double ph = 1.0 - (1.0 - A.phi[i]) / Jd;            // Eq. 16
  const double Sr = swrc(P, Jn, ph, A.s[i]);                // Eq. 15
  A.J_out[i] = Jn;
  A.vol_out[i] = Vn;
  A.phi_out[i] = ph;
  A.Sr_out[i] = Sr;
  A.mass_out[i] = (P.rho_s * (1.0 - ph) + P.rho_w * Sr * ph) * Vn;   // Eq. 48
  A.pk[i] = apparent_pc(P, A.pc[i]);
  A.pk[n + i] = Vp > 0.0 ? 1.0 / Vp : 0.0;
}

// Point kinematics with four lanes per point (a DPP quad): each lane walks
// every fourth member of the family (the loads of four members in flight at
// once), the quad adds its partial sums, and its first lane updates the point.
// A workgroup holds 64 consecutive points; the workgroups of one XCD take a
// contiguous range of them.  (One lane per point left only two waves per SIMD
// on C1, too few to hide the gathers' latency.)
constexpr int kKinLanes = 4;
constexpr int kKinPoints = 256 / kKinLanes;                  // points per workgroup
__global__ __launch_bounds__(256) void k_point_kin_quad(BondArgs A, DevParams P, int64_t per) {
  const int64_t blk = xcd_point(blockIdx.x, per);
  const int sub = threadIdx.x & (kKinLanes - 1);
  const int64_t i = blk * kKinPoints + threadIdx.x / kKinLanes;
  if (i >= A.n) return;                                       // whole quads
  const int64_t n = A.n;
  const int64_t b0 = A.row[i], b1 = A.row[i + 1];
  const double xi0 = A.x[i], xi1 = A.x[n + i], xi2 = A.x[2 * n + i];
  const double vi0 = A.vh[i], vi1 = A.vh[n + i], vi2 = A.vh[2 * n + i];
  double Kp[6] = {0, 0, 0, 0, 0, 0}, Np[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Vp = 0.0;
  const double4* xv = reinterpret_cast<const double4*>(A.xv);
  for (int64_t s0 = b0 + sub; s0 < b1; s0 += 4 * kKinLanes) {
    double4 pa[4], pb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t s = s0 + kKinLanes * u < b1 ? s0 + kKinLanes * u : s0;
      const int32_t k = A.col[s];
      pa[u] = xv[2 * (int64_t)k];
      pb[u] = xv[2 * (int64_t)k + 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (s0 + kKinLanes * u >= b1) break;
      const double z0 = pa[u].x - xi0, z1 = pa[u].y - xi1, z2 = pa[u].z - xi2;
      const double y0 = pb[u].x - vi0, y1 = pb[u].y - vi1, y2 = pb[u].z - vi2;
      const double V = pa[u].w;
      const double w0 = V * z0, w1 = V * z1, w2 = V * z2;
      Kp[0] += w0 * z0; Kp[1] += w1 * z1; Kp[2] += w2 * z2;
      Kp[3] += w1 * z2; Kp[4] += w0 * z2; Kp[5] += w0 * z1;
      Np[0] += y0 * w0; Np[1] += y0 * w1; Np[2] += y0 * w2;
      Np[3] += y1 * w0; Np[4] += y1 * w1; Np[5] += y1 * w2;
      Np[6] += y2 * w0; Np[7] += y2 * w1; Np[8] += y2 * w2;
      Vp += V;
    }
  }
  // quad sums: every lane of the quad ends with the totals
  auto quad_sum = [](double v) {
    v += dpp_d<kDppXor1, 0xF>(v);
    return v + dpp_d<kDppXor2, 0xF>(v);
  };
#pragma unroll
  for (int k = 0; k < 6; ++k) Kp[k] = quad_sum(Kp[k]);
#pragma unroll
  for (int k = 0; k < 9; ++k) Np[k] = quad_sum(Np[k]);
  Vp = quad_sum(Vp);
  if (sub == 0) point_update(A, P, i, (int)(b1 - b0), Kp, Np, Vp);
}

// The standard correspondence model (Eqs. 12-14): one wave per point forms
// the full-horizon sums and the point update, then every lane updates the
// point stress from L_i by the return map and writes T_ij = (sigma_i + S_r s 1)
// K_i^{-1} zeta_ij for its bonds of the point.
template <class TS>
__global__ __launch_bounds__(256) void k_point_kin_standard(BondArgs A, DevParams P) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t n = A.n;
  const XcdWalk W = xcd_walk(n, 4);
  int c_deg = 0, c_pl = 0, c_nc = 0, c_mx = 0;          // lane 0
  for (int64_t i = W.first; i < W.end; i += W.stride) {
    const int64_t b0 = A.row[i], b1 = A.row[i + 1];
    const double xi0 = A.x[i], xi1 = A.x[n + i], xi2 = A.x[2 * n + i];
    const double vi0 = A.vh[i], vi1 = A.vh[n + i], vi2 = A.vh[2 * n + i];
    double Kp[6] = {0, 0, 0, 0, 0, 0}, Np[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Vp = 0.0;
    for (int64_t s = b0 + lane; s < b1; s += kWave) {
      const int32_t k = A.col[s];
      const double4 pa = reinterpret_cast<const double4*>(A.xv)[2 * (int64_t)k];
      const double4 pb = reinterpret_cast<const double4*>(A.xv)[2 * (int64_t)k + 1];
      const double z0 = pa.x - xi0, z1 = pa.y - xi1, z2 = pa.z - xi2;
      const double y0 = pb.x - vi0, y1 = pb.y - vi1, y2 = pb.z - vi2;
      const double V = pa.w;
      const double w0 = V * z0, w1 = V * z1, w2 = V * z2;
      Kp[0] += w0 * z0; Kp[1] += w1 * z1; Kp[2] += w2 * z2;
      Kp[3] += w1 * z2; Kp[4] += w0 * z2; Kp[5] += w0 * z1;
      Np[0] += y0 * w0; Np[1] += y0 * w1; Np[2] += y0 * w2;
      Np[3] += y1 * w0; Np[4] += y1 * w1; Np[5] += y1 * w2;
      Np[6] += y2 * w0; Np[7] += y2 * w1; Np[8] += y2 * w2;
      Vp += V;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) Kp[k] = wave_sum(Kp[k]);
#pragma unroll
    for (int k = 0; k < 9; ++k) Np[k] = wave_sum(Np[k]);
    Vp = wave_sum(Vp);
    if (lane == 0) point_update(A, P, i, (int)(b1 - b0), Kp, Np, Vp);
    {
      // every lane holds the wave totals and forms the point update itself
      const int nf = (int)(b1 - b0);
      double Ki[6] = {0, 0, 0, 0, 0, 0};
      const bool ok = shape_inverse(P.plane != 0, Kp, nf, Ki);
      double sg[6], pcn = A.pc[i], pco = pcn;
      for (int k = 0; k < 6; ++k) sg[k] = A.sig[k][i];
      double so[6] = {sg[0], sg[1], sg[2], sg[3], sg[4], sg[5]};
      if (ok) {
        double KiF[9], L[9];
        sym_full(Ki, KiF);
        mat3_mul(Np, KiF, L);
        const double h = A.dt_inc;
        if (h != 0.0) {
          const double de[6] = {h * L[0], h * L[4], h * L[8], h * 0.5 * (L[5] + L[7]), h * 0.5 * (L[2] + L[6]),
                                h * 0.5 * (L[1] + L[3])};
          int it = return_map(P, h, sg, pcn, de, so, &pco);
          if (lane == 0) {
            if (it < 0) { ++c_nc; it = P.newton_maxit; }
            if (it > 0) ++c_pl;
            c_mx = c_mx > it ? c_mx : it;
          }
        }
      } else if (lane == 0) {
        c_deg += nf;
      }
      if (lane == 0) {
        for (int k = 0; k < 6; ++k) A.sig_out[k][i] = so[k];
        A.pc_out[i] = pco;
      }
      // total stress sigma_i + S_r s 1 (Eq. 14 with p_w = -s) times K_i^{-1}
      double SK[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      if (ok) {
        const double ps = A.Sr_out[i] * A.s[i];
        const double Q[6] = {so[0] + ps, so[1] + ps, so[2] + ps, so[3], so[4], so[5]};
        double QF[9], KiF[9];
        sym_full(Q, QF);
        sym_full(Ki, KiF);
        mat3_mul(QF, KiF, SK);
      }
      Quad<TS>* T4 = reinterpret_cast<Quad<TS>*>(A.T);
      for (int64_t s = b0 + lane; s < b1; s += kWave) {
        const int32_t k = A.col[s];
        const double4 pa = reinterpret_cast<const double4*>(A.xv)[2 * (int64_t)k];
        const double z0 = pa.x - xi0, z1 = pa.y - xi1, z2 = pa.z - xi2;
        T4[s] = Quad<TS>{{(TS)(SK[0] * z0 + SK[1] * z1 + SK[2] * z2), (TS)(SK[3] * z0 + SK[4] * z1 + SK[5] * z2),
                          (TS)(SK[6] * z0 + SK[7] * z1 + SK[8] * z2), (TS)0}};
      }
    }
  }
  if (lane == 0) {
    if (c_deg) ctr_add(A.ctr, C_DEGEN, (unsigned long long)c_deg);
    if (c_pl) ctr_add(A.ctr, C_PLASTIC, (unsigned long long)c_pl);
    if (c_nc) ctr_add(A.ctr, C_NOCONV, (unsigned long long)c_nc);
    if (c_mx) ctr_max(A.ctr, C_MAXNEWTON, (unsigned long long)c_mx);
  }
}

// History carried on the bonds: the start states of the new families' bonds,
// copied (the reverse step's input).  One wave per point, lanes over its
// bonds; a bond found (binary search) in the point's row of the previous
// families keeps its state, a new bond starts from the point history
// (sigma_i, p_c,i).  Rows of both are ascending.
__global__ __launch_bounds__(256) void k_hist_carry(int64_t n, const int64_t* __restrict__ row,
                                                    const int32_t* __restrict__ col,
                                                    const int64_t* __restrict__ hrow,
                                                    const int32_t* __restrict__ hcol, int have, int max_f,
                                                    const double* __restrict__ hold, double* __restrict__ hcur,
                                                    ulppm_state S) {
  // one wave per point: the point's previous row is staged in LDS (at most
  // max_f sorted columns) and every new bond binary-searches it there
  extern __shared__ int32_t s_hcol[];
  int32_t* rowc = s_hcol + (threadIdx.x / kWave) * (size_t)max_f;
  const int lane = threadIdx.x & (kWave - 1);
  const XcdWalk W = xcd_walk(n, 4);
  const double4* ho = reinterpret_cast<const double4*>(hold);
  double4* hc = reinterpret_cast<double4*>(hcur);
  for (int64_t i = W.first; i < W.end; i += W.stride) {
    const int64_t b0 = row[i], b1 = row[i + 1];
    const int64_t h0 = have ? hrow[i] : 0;
    const int nh = have ? (int)min<int64_t>(hrow[i + 1] - h0, max_f) : 0;
    for (int t = lane; t < nh; t += kWave) rowc[t] = hcol[h0 + t];
    __builtin_amdgcn_wave_barrier();               // this wave's row is in place (LDS is in order per wave)
    for (int64_t s = b0 + lane; s < b1; s += kWave) {
      const int32_t j = col[s];
      int lo = 0, hi = nh;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rowc[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      if (lo < nh && rowc[lo] == j) {
        hc[2 * s] = ho[2 * (h0 + lo)];
        hc[2 * s + 1] = ho[2 * (h0 + lo) + 1];
      } else {
        hc[2 * s] = double4{S.sig[0][i], S.sig[1][i], S.sig[2][i], S.sig[3][i]};
        hc[2 * s + 1] = double4{S.sig[4][i], S.sig[5][i], S.pc[i], 0.0};
      }
    }
    __builtin_amdgcn_wave_barrier();               // every lane is done with the row before the next
  }
}

// The forward's carry as a map: for every bond of the new families its slot
// in the previous families (-1 for a bond that enters), so that the bond
// kernel reads the old states directly.  One wave per point, as k_hist_carry.
__global__ __launch_bounds__(256) void k_hist_map(int64_t n, const int64_t* __restrict__ row,
                                                  const int32_t* __restrict__ col, const int64_t* __restrict__ hrow,
                                                  const int32_t* __restrict__ hcol, int have, int max_f,
                                                  int64_t* __restrict__ hmap) {
  extern __shared__ int32_t s_hcol[];
  int32_t* rowc = s_hcol + (threadIdx.x / kWave) * (size_t)max_f;
  const int lane = threadIdx.x & (kWave - 1);
  const XcdWalk W = xcd_walk(n, 4);
  for (int64_t i = W.first; i < W.end; i += W.stride) {
    const int64_t b0 = row[i], b1 = row[i + 1];
    const int64_t h0 = have ? hrow[i] : 0;
    const int nh = have ? (int)min<int64_t>(hrow[i + 1] - h0, max_f) : 0;
    for (int t = lane; t < nh; t += kWave) rowc[t] = hcol[h0 + t];
    __builtin_amdgcn_wave_barrier();
    for (int64_t s = b0 + lane; s < b1; s += kWave) {
      const int32_t j = col[s];
      int lo = 0, hi = nh;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rowc[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      hmap[s] = (lo < nh && rowc[lo] == j) ? h0 + lo : -1;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Families of the last step, kept with the bond states they order.
__global__ void k_hist_keep(int64_t n, const int64_t* __restrict__ row, const int32_t* __restrict__ col,
                            int64_t* __restrict__ hrow, int32_t* __restrict__ hcol) {
  const int64_t nb = row[n];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e <= n; e += (int64_t)gridDim.x * blockDim.x)
    hrow[e] = row[e];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nb; e += (int64_t)gridDim.x * blockDim.x)
    hcol[e] = col[e];
}

// Reverse of k_hist_carry: a carried bond hands the adjoint of its start
// state back to the bond it came from (hbar0, in the previous families'
// order, zero elsewhere); a new bond, which started from its point, adds it
// to the adjoint of the point's history (sigb, pcb).  One wave per point.
__global__ __launch_bounds__(256) void k_adj_hist_carry(int64_t n, const int64_t* __restrict__ row,
                                                        const int32_t* __restrict__ col,
                                                        const int64_t* __restrict__ hrow,
                                                        const int32_t* __restrict__ hcol, int have, int max_f,
                                                        const double* __restrict__ hb0s, double* __restrict__ hbar0,
                                                        double* __restrict__ sigb, double* __restrict__ pcb) {
  extern __shared__ int32_t s_hcol[];
  int32_t* rowc = s_hcol + (threadIdx.x / kWave) * (size_t)max_f;
  const int lane = threadIdx.x & (kWave - 1);
  const XcdWalk W = xcd_walk(n, 4);
  for (int64_t i = W.first; i < W.end; i += W.stride) {
    const int64_t b0 = row[i], b1 = row[i + 1];
    const int64_t h0 = have ? hrow[i] : 0;
    const int nh = have ? (int)min<int64_t>(hrow[i + 1] - h0, max_f) : 0;
    for (int t = lane; t < nh; t += kWave) rowc[t] = hcol[h0 + t];
    __builtin_amdgcn_wave_barrier();
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t s = b0 + lane; s < b1; s += kWave) {
      const int32_t j = col[s];
      int lo = 0, hi = nh;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rowc[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      const double* src = hb0s + 8 * s;
      if (lo < nh && rowc[lo] == j) {
        double* dst = hbar0 + 8 * (h0 + lo);
        for (int k = 0; k < 7; ++k) dst[k] = src[k];
      } else {
        for (int k = 0; k < 7; ++k) acc[k] += src[k];
      }
    }
    for (int k = 0; k < 7; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0) {
      for (int k = 0; k < 6; ++k) sigb[k * n + i] += acc[k];
      pcb[i] += acc[6];
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------- bond kernel, MFMA sums --
//
// The masked sums of pass 1 (sub-horizon shape tensor, velocity-gradient
// sum and volume, Eqs. 22-23, 25, 55, 57) and of pass 2 (force states,
// Eqs. 27, 31, 35) are both products of the family's 0/1 membership matrix
// B with a per-member feature matrix:
//   pass 1: [K_j | N_j | Vs_j] = sum_k B_jk V_k [zeta_k zeta_k^T (6), ydot_k zeta_k^T (9), 1]
//   pass 2: A_k = sum_j B_kj M_j  (9), then T_ik = A_k zeta_ik.
// They run on the matrix cores as 16x16x4 products (rows: sub-horizons or
// members, K: members, N: 16 features), FP64 or FP32 (mixed precision),
// while the VALU evaluates the exact FP64 membership predicate that forms
// the 0/1 operand.  Lane layout of the 16x16x4 products (64 lanes, checked
// on gfx950): A[i][k] in lane i + 16 k, B[k][f] in lane f + 16 k; the result
// D[i][f] sits in lane f + 16 (i / 4), element i % 4, for FP32 and in lane
// f + 16 (i % 4), element i / 4, for FP64.
//
// Membership bits: for row r and column block c (64 members), word
// sb[r * nw + c] holds in bit 16 q + s the membership of member 64 c + 4 s + q,
// so that the lane that tests (r, 4 s + q) owns one 16-bit quarter.

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 2 p + (this lane's bit of the lane mask m): one add with carry, the mask
// as the carry-in.  Written out because the compiler forms the sum from a
// select and a shift-or.
__device__ __forceinline__ unsigned shift_in(unsigned p, unsigned long long m) {
  unsigned r;
  asm("v_addc_co_u32 %0, %1, %2, %2, %1" : "=v"(r), "+s"(m) : "v"(p));
  return r;
}

template <class Acc>
struct Mma;
template <>
struct Mma<double> {
  using V = v4d;
  static __device__ __forceinline__ V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of result element r in lane group q (lane / 16)
  static __device__ __forceinline__ int row(int q, int r) { return 4 * r + q; }
};
template <>
struct Mma<float> {
  using V = v4f;
  static __device__ __forceinline__ V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; }
};

#ifndef ULPPM_TILE_BATCH
#define ULPPM_TILE_BATCH 4
#endif
constexpr int kTileBatch = ULPPM_TILE_BATCH;   // 16-row tiles a wave carries through one sweep over the members
static_assert(kTileBatch >= 1 && kTileBatch <= 4, "tile_slots dispatches 1 to 4 tiles");

// Run f(t0, NB) for the NB = min(nb, kTileBatch) tile slots t0, t0 + waves, ...
// left to one wave, NB a compile-time constant.
template <class F>
__device__ __forceinline__ void tile_slots(int nb, int t0, F&& f) {
  if (kTileBatch >= 4 && nb >= 4) f(t0, std::integral_constant<int, 4>{});
  else if (kTileBatch >= 3 && nb >= 3) f(t0, std::integral_constant<int, 3>{});
  else if (kTileBatch >= 2 && nb >= 2) f(t0, std::integral_constant<int, 2>{});
  else f(t0, std::integral_constant<int, 1>{});
}
constexpr size_t kCuLds = 160 * 1024;       // LDS of one CU
constexpr size_t kBondStaticLds = 512;      // headroom for static LDS in the occupancy estimate

// Member slots of the staged records: the family padded to whole 16-row
// tiles, plus (mixed precision) the quad the member loop loads one step
// ahead; in FP64 that last, unused look-ahead load falls on the sums that
// follow the records.  Padding slots hold positions outside every horizon
// (no membership) and zero features.
template <class Acc>
__host__ __device__ constexpr int bond_mx_slots(int max_f) {
  return ((max_f + 15) & ~15) + (sizeof(Acc) == 8 ? 0 : 4);
}
// Rows of the 16 member sums: the family capacity rounded up to whole groups
// of four, which pass 2 reads without range checks.
__host__ __device__ constexpr int bond_mx_rows(int max_f) { return (max_f + 3) & ~3; }
// Bytes of one member slot.  FP64: the record {x_k, V_k, ydot_ik, 1}, with
// zeta_ik = x_k - x_i formed where it is needed.  Mixed: (x_k, V_k) in FP64 for
// the membership test beside the record {zeta_ik, V_k, ydot_ik, 1} in FP32.
template <class Acc>
__host__ __device__ constexpr size_t bond_mx_slot_bytes() {
  return sizeof(Acc) == 8 ? 8 * sizeof(double) : sizeof(Quad<double>) + 8 * sizeof(Acc);
}
// Rows of the closing reduction (one double per thread each): the point
// history sums (8), the own force-state sums (3) and four counters.
constexpr int kCloseRows = 15;
template <class Acc>
__host__ __device__ constexpr size_t bond_mx_lds_bytes(int max_f, int nt) {
  // the member slots, the 16 sums and the membership bits per member.  The
  // closing reduction reuses the space for 16 rows of one double per thread
  // and the per-wave maxima after them.  The kernel has no static LDS: at
  // family capacity 128 the FP64 workgroup needs 26 KB, and six fit a CU.
  return (size_t)bond_mx_slots<Acc>(max_f) * bond_mx_slot_bytes<Acc>() +
                 (size_t)bond_mx_rows(max_f) * 16 * sizeof(Acc) +
                 (size_t)max_f * ((max_f + 63) / 64) * sizeof(unsigned long long) >
             16 * (size_t)nt * sizeof(double) + 128
         ? (size_t)bond_mx_slots<Acc>(max_f) * bond_mx_slot_bytes<Acc>() +
               (size_t)bond_mx_rows(max_f) * 16 * sizeof(Acc) +
               (size_t)max_f * ((max_f + 63) / 64) * sizeof(unsigned long long)
         : 16 * (size_t)nt * sizeof(double) + 128;
}

// Feature f of member k (pass 1, B operand): V_k a_f b_f from the record
// {zeta0, zeta1, zeta2, V, ydot0, ydot1, ydot2, 1}.
__host__ __device__ constexpr int feat_a(int f) {
  return f < 3 ? f : f == 3 ? 1 : f < 6 ? 0 : f < 15 ? 4 + (f - 6) / 3 : 7;
}
__host__ __device__ constexpr int feat_b(int f) {
  return f < 3 ? f : f == 3 ? 2 : f == 4 ? 2 : f == 5 ? 1 : f < 15 ? (f - 6) % 3 : 7;
}

// NT threads per workgroup (one point): 128 for 3D families of ~100, 64 when
// every family fits one wave (plane strain).  MW: waves per SIMD the instance
// is compiled for, chosen on the host from the workgroups the LDS of the
// family capacity lets a CU hold (bond_waves).  The kernel waits on LDS and on
// dependent FP64 chains, so a wave more gains more than it loses to spilled
// registers; an instance compiled for more waves than the LDS admits would
// only spill.  LinP: the run's apparent pre-consolidation is linear (Eq. 45
// with b1 = 0, b2 = 1), which takes the general power, the register peak of
// the return map, out of the instance.
template <class Acc, bool Hist, bool LinP, int NT, int MW>
__global__ __launch_bounds__(NT, MW)
void k_bond_mx(BondArgs A, DevParams P) {
  constexpr int kBondThreads = NT, kBondWaves = NT / kWave;
  using TS = Acc;
  using MM = Mma<Acc>;
  using V4 = typename MM::V;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t i = xcd_point(blockIdx.x, A.per);
  if (i >= A.n) return;                           // uniform per block
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int mf = A.max_f;
  const int64_t n = A.n;
  const int64_t b0 = A.row[i];
  const int nf = (int)(A.row[i + 1] - b0);
  const int nw = (mf + 63) / 64;                   // membership words per row
  // The membership test of Eq. 22 compares |x_k - x_j| from the positions.
  // FP64: one record {x_k, V_k, ydot_ik, 1} per slot, zeta_ik = x_k - x_i
  // formed where it is needed.  Mixed: (x_k, V_k) in FP64 beside the record
  // {zeta_ik, V_k, ydot_ik, 1} in FP32 (zeta formed in FP64, then rounded).
  constexpr bool kF64 = sizeof(Acc) == 8;
  const int mfp = bond_mx_slots<Acc>(mf);
  Quad<double>* sX = reinterpret_cast<Quad<double>*>(smem_raw);        // mixed only
  Acc* sR = kF64 ? reinterpret_cast<Acc*>(smem_raw) : reinterpret_cast<Acc*>(sX + mfp);
  Acc* sKN = sR + 8 * (size_t)mfp;                                     // 16 per member: K, N, Vs, then M_j
  unsigned long long* sb = reinterpret_cast<unsigned long long*>(sKN + 16 * (size_t)bond_mx_rows(mf));
  unsigned short* sq = reinterpret_cast<unsigned short*>(sb);
  Quad<TS>* const T4 = reinterpret_cast<Quad<TS>*>(A.T);

  const double xi0 = A.x[i], xi1 = A.x[n + i], xi2 = A.x[2 * n + i];
  const double vi0 = A.vh[i], vi1 = A.vh[n + i], vi2 = A.vh[2 * n + i];
  // position of slot m for the membership test
  auto pos = [&](int m) -> Quad<double> {
    if constexpr (kF64) return reinterpret_cast<const Quad<double>*>(sR)[2 * m];
    else return sX[m];
  };

  // Stage the family of i: x_k and V_k (FP64, for the exact predicate),
  // ydot_ik, and in mixed precision zeta_ik formed in FP64 before rounding.
  for (int m = tid; m < nf; m += kBondThreads) {
    const int32_t k = A.col[b0 + m];
    const double4 pa = reinterpret_cast<const double4*>(A.xv)[2 * (int64_t)k];
    const double4 pb = reinterpret_cast<const double4*>(A.xv)[2 * (int64_t)k + 1];
    const double Vk = pa.w;
    const double y0 = pb.x - vi0, y1 = pb.y - vi1, y2 = pb.z - vi2;
    Acc* rec = sR + 8 * (size_t)m;
    if constexpr (kF64) {
      rec[0] = pa.x; rec[1] = pa.y; rec[2] = pa.z;
    } else {
      sX[m] = Quad<double>{{pa.x, pa.y, pa.z, Vk}};
      rec[0] = (Acc)(pa.x - xi0); rec[1] = (Acc)(pa.y - xi1); rec[2] = (Acc)(pa.z - xi2);
    }
    rec[3] = (Acc)Vk;
    rec[4] = (Acc)y0; rec[5] = (Acc)y1; rec[6] = (Acc)y2; rec[7] = (Acc)1;
  }
  const int ntile = (nf + 15) >> 4;
  const int nks = (nf + 3) >> 2;
  const int nblk = (nks + 15) >> 4;               // bit words per row written by pass 1
  // padding slots up to whole tiles (and the look-ahead quad in mixed
  // precision): positions outside every horizon fail every membership test
  // (FP64: 1e6 m away, so that the features V a b stay finite and vanish
  // with V = 0; mixed: infinity, beside zero features), so the member loop
  // needs no range checks
  for (int m = nf + tid; m < (kF64 ? 16 * ntile : max(16 * ntile, 4 * nks + 4)); m += kBondThreads) {
    Acc* rec = sR + 8 * (size_t)m;
#pragma unroll
    for (int q = 0; q < 8; ++q) rec[q] = (Acc)0;
    if constexpr (kF64) {
      rec[0] = xi0 + 1e6; rec[1] = xi1 + 1e6; rec[2] = xi2 + 1e6;
    } else {
      sX[m] = Quad<double>{{INFINITY, INFINITY, INFINITY, 0.0}};
    }
  }
  __syncthreads();
  const double d2 = P.d2;

  // ---- pass 1: membership matrix x features on the matrix cores.  Tiles
  // past the family (and rows past nf) carry zero operands; everything in
  // the member loop is branch-free so that tests and products interleave.
  {
    const int fa = feat_a(r16), fb = feat_b(r16);
    // the FP64 records hold x_k: the zeta features subtract x_i
    const double xi[3] = {xi0, xi1, xi2};
    const Acc oa = kF64 && fa < 3 ? (Acc)xi[fa < 3 ? fa : 0] : (Acc)0;
    const Acc ob = kF64 && fb < 3 ? (Acc)xi[fb < 3 ? fb : 0] : (Acc)0;
    // NB tile slots t0, t0 + kBondWaves, ... of one wave, all inside the family
    auto tiles = [&](int t0, auto nbc) {
      constexpr int NB = decltype(nbc)::value;
      double xj[NB][3];
      bool jv[NB];
      int jrow[NB];
      V4 acc[NB];
      unsigned piece[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        jrow[b] = (t0 + kBondWaves * b) * 16 + r16;
        jv[b] = jrow[b] < nf;
        const Quad<double> q = pos(jrow[b]);         // a padding slot past the family
        xj[b][0] = q.v[0]; xj[b][1] = q.v[1]; xj[b][2] = q.v[2];
        acc[b] = V4{0, 0, 0, 0};
        piece[b] = 0u;
      }
      // Member data of step ks: position and the three feature factors.
      struct StepData {
        Quad<double> x;
        Acc ra, rb, rv;
      };
      auto load = [&](int ks) {
        const int k = 4 * ks + q4;
        const Acc* rec = sR + 8 * (size_t)k;
        return StepData{pos(k), rec[fa] - oa, rec[fb] - ob, rec[3]};
      };
      // The bits of a piece are shifted in (2 piece + in: one add with carry),
      // so step s of the piece's c steps sits at bit c - 1 - s; the store
      // reverses them into bit s.
      auto step = [&](int ks, const StepData& m) {
        const Acc bval = m.ra * m.rb * m.rv;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const bool in = within(xj[b][0], xj[b][1], xj[b][2], m.x.v[0], m.x.v[1], m.x.v[2], d2);
          piece[b] = shift_in(piece[b], __ballot(in));
          acc[b] = MM::run(in ? (Acc)1 : (Acc)0, bval, acc[b]);
        }
        if ((ks & 15) == 15 || ks == nks - 1) {
          const unsigned up = 15 - (ks & 15);         // 16 - c
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const unsigned bits = __builtin_bitreverse32(piece[b] << up) >> 16;
            if (jv[b]) sq[((size_t)jrow[b] * nw + (ks >> 4)) * 4 + q4] = (unsigned short)bits;
            piece[b] = 0u;
          }
        }
      };
      // Two steps per iteration, each step's data loaded one step ahead into
      // alternating registers (no copies between iterations).  The last
      // look-ahead reads slot 4 nks + q4 at most, as the member loop always
      // has (a padding slot, or in FP64 the sums that follow the records).
      StepData ma = load(0);
      int ks = 0;
      for (; ks + 1 < nks; ks += 2) {
        const StepData mb = load(ks + 1);
        step(ks, ma);
        ma = load(ks + 2);
        step(ks + 1, mb);
      }
      if (ks < nks) step(ks, ma);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int t = t0 + kBondWaves * b;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = t * 16 + MM::row(q4, r);
          if (j < nf) sKN[16 * (size_t)j + r16] = acc[b][r];
        }
      }
    };
    for (int t0 = wid; t0 < ntile; t0 += kBondWaves * kTileBatch) {
      const int nb = (ntile - t0 + kBondWaves - 1) / kBondWaves;     // slots left for this wave
      tile_slots(nb, t0, tiles);
    }
  }
  __syncthreads();

  // ---- per-bond tail: one lane per bond (i,j); the per-point values of
  // this step (point kinematics) are loaded here, not kept through pass 1
  const double Sr_i = A.Sr_out[i], Pn_i = A.pk[i], iVh = A.pk[n + i];
  const double s_i = A.s[i];
  double sig_i[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) sig_i[k] = A.sig[k][i];
  const double pc_i = A.pc[i];
  double hs[6] = {0, 0, 0, 0, 0, 0}, hpc = 0.0, hw = 0.0;
  int n_deg = 0, n_pl = 0, n_nc = 0, n_trip = 0, mx = 0;
  // One lane per bond.  The lane's sums above start at zero for its first
  // bond, so nothing is carried through that bond's return map (the
  // kernel's register peak).  Families wider than the workgroup take
  // further bonds per lane; the sums are then carried as wave totals,
  // which are uniform, and handed back to lane 0 for the closing reduction.
  auto tail = [&](const int m) {
    Acc* kn = sKN + 16 * (size_t)m;
    int ns = 0;
    for (int c = 0; c < nblk; ++c) ns += __popcll(sb[(size_t)m * nw + c]);
    n_trip += ns;
    // FP64 from here on: inversion, gradient, return map, force state.
    const int64_t slot = b0 + m;
    // K_ij^{-1} (symmetric: xx, yy, zz, xy, xz, yz) from the sums in LDS.  The
    // mixed-precision instances, compiled for four waves per SIMD, form it
    // again after the return map (their register peak) rather than keep it
    // through it; the recomputation is bit-identical, and the empty asm keeps
    // the compiler from reusing the first reads.  The FP64 instances keep it.
    auto kinv = [&](double* I) -> bool {
      asm volatile("" ::: "memory");
      const double a = kn[0], b = kn[1], c = kn[2], d = kn[3], e = kn[4], f = kn[5];
      if (P.plane) {                                            // x-z block (plane strain)
        const double d2 = a * c - e * e, tr = (a + c) / 2.0;
        const double id = 1.0 / d2;
        I[0] = c * id; I[2] = a * id; I[4] = -e * id;
        I[1] = I[3] = I[5] = 0.0;
        return ns >= 2 && d2 > 1e-12 * tr * tr;
      }
      const double dK = det3s(a, b, c, d, e, f);
      const double tk = (a + b + c) / 3.0;
      const double idK = 1.0 / dK;
      I[0] = (b * c - d * d) * idK; I[1] = (a * c - e * e) * idK; I[2] = (a * b - f * f) * idK;
      I[3] = (d * e - f * c) * idK; I[4] = (f * d - b * e) * idK; I[5] = (e * f - a * d) * idK;
      return ns >= 3 && dK > 1e-12 * tk * tk * tk;
    };
    double Ki[6];
    const bool ok = kinv(Ki);
    // history on the bonds: the state the bond starts from
    double sg0[6] = {0, 0, 0, 0, 0, 0}, pc0 = 0.0;
    if constexpr (Hist) {
      const int64_t src = A.hmap[slot];
      if (src >= 0) {
        const double4 ha = reinterpret_cast<const double4*>(A.hist_old)[2 * src];
        const double4 hb = reinterpret_cast<const double4*>(A.hist_old)[2 * src + 1];
        sg0[0] = ha.x; sg0[1] = ha.y; sg0[2] = ha.z; sg0[3] = ha.w; sg0[4] = hb.x; sg0[5] = hb.y;
        pc0 = hb.z;
      } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) sg0[k] = sig_i[k];
        pc0 = pc_i;
      }
    }
    if (__builtin_expect(!ok, 0)) {                             // degenerate: inactive bond
      ++n_deg;
#pragma unroll
      for (int q = 0; q < 9; ++q) kn[q] = (Acc)0;
      if (P.force_mode == ULPPM_FORCE_EQ51) T4[slot] = Quad<TS>{{(TS)0, (TS)0, (TS)0, (TS)0}};
      if constexpr (Hist) {                                     // an inactive bond keeps its state
        reinterpret_cast<double4*>(A.hist)[2 * slot] = double4{sg0[0], sg0[1], sg0[2], sg0[3]};
        reinterpret_cast<double4*>(A.hist)[2 * slot + 1] = double4{sg0[4], sg0[5], pc0, 0.0};
      }
      return;
    }
    double N[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) N[q] = (double)kn[6 + q];
    double L[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      L[3 * r + 0] = N[3 * r] * Ki[0] + N[3 * r + 1] * Ki[3] + N[3 * r + 2] * Ki[4];
      L[3 * r + 1] = N[3 * r] * Ki[3] + N[3 * r + 1] * Ki[1] + N[3 * r + 2] * Ki[5];
      L[3 * r + 2] = N[3 * r] * Ki[4] + N[3 * r + 1] * Ki[5] + N[3 * r + 2] * Ki[2];
    }
    const double varpi = (double)kn[15] * iVh;                  // Eq. 55
    const double h = A.dt_inc;
    const double de[6] = {h * L[0], h * L[4], h * L[8], h * 0.5 * (L[5] + L[7]), h * 0.5 * (L[2] + L[6]),
                          h * 0.5 * (L[1] + L[3])};              // Eqs. 26, 59
    double sgb[6], pcb;
    if constexpr (!Hist) {                                      // bonds start from the point history
      if (h == 0.0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) sgb[k] = sig_i[k];
        pcb = pc_i;
      } else {
        int it = return_map_pn<LinP>(P, h, sig_i, pc_i, Pn_i, de, sgb, &pcb);
        if (it < 0) { ++n_nc; it = P.newton_maxit; }
        if (it > 0) ++n_pl;
        mx = mx > it ? mx : it;
      }
    } else {                                                    // each bond starts from its own state
      if (h == 0.0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) sgb[k] = sg0[k];
        pcb = pc0;
      } else {
        int it = return_map_pn<LinP>(P, h, sg0, pc0, apparent_pc<LinP>(P, pc0), de, sgb, &pcb);
        if (it < 0) { ++n_nc; it = P.newton_maxit; }
        if (it > 0) ++n_pl;
        mx = mx > it ? mx : it;
      }
      reinterpret_cast<double4*>(A.hist)[2 * slot] = double4{sgb[0], sgb[1], sgb[2], sgb[3]};
      reinterpret_cast<double4*>(A.hist)[2 * slot + 1] = double4{sgb[4], sgb[5], pcb, 0.0};
    }
    if constexpr (!kF64) kinv(Ki);
    const double ixx = Ki[0], iyy = Ki[1], izz = Ki[2], ixy = Ki[3], ixz = Ki[4], iyz = Ki[5];
    // Total bond stress sigma_ij + Sr_i s_i 1 (Eq. 32 with p_w = -s) times K_ij^{-1}.
    const double ps = Sr_i * s_i;
    const double S00 = sgb[0] + ps, S11 = sgb[1] + ps, S22 = sgb[2] + ps;
    const double SK[9] = {S00 * ixx + sgb[5] * ixy + sgb[4] * ixz, S00 * ixy + sgb[5] * iyy + sgb[4] * iyz,
                          S00 * ixz + sgb[5] * iyz + sgb[4] * izz, sgb[5] * ixx + S11 * ixy + sgb[3] * ixz,
                          sgb[5] * ixy + S11 * iyy + sgb[3] * iyz, sgb[5] * ixz + S11 * iyz + sgb[3] * izz,
                          sgb[4] * ixx + sgb[3] * ixy + S22 * ixz, sgb[4] * ixy + sgb[3] * iyy + S22 * iyz,
                          sgb[4] * ixz + sgb[3] * iyz + S22 * izz};
    const double Vj = kF64 ? (double)sR[8 * (size_t)m + 3] : sX[m].v[3];
    if (P.force_mode == ULPPM_FORCE_EQ51) {
      // Eq. 51 as printed: T_ij = varpi (sigma_ij + Sr s 1) K_ij^{-1} zeta_ij.
      const double zx = kF64 ? sR[8 * (size_t)m] - xi0 : (double)sR[8 * (size_t)m];
      const double zy = kF64 ? sR[8 * (size_t)m + 1] - xi1 : (double)sR[8 * (size_t)m + 1];
      const double zz = kF64 ? sR[8 * (size_t)m + 2] - xi2 : (double)sR[8 * (size_t)m + 2];
      const double t0 = varpi * (SK[0] * zx + SK[1] * zy + SK[2] * zz),
                   t1 = varpi * (SK[3] * zx + SK[4] * zy + SK[5] * zz),
                   t2 = varpi * (SK[6] * zx + SK[7] * zy + SK[8] * zz);
      if constexpr (kF64) {
        // With the own sums kept, the record holds V_i T_ij (as in the
        // conjugate path) and the bond's row, no longer read, T_ij V_j: the
        // lane sums its rows after the last bond, so that nothing is carried
        // through the return maps of its further bonds.
        const double sc = A.fown ? A.vol_n[i] : 1.0;
        T4[slot] = Quad<TS>{{(TS)(sc * t0), (TS)(sc * t1), (TS)(sc * t2), (TS)0}};
        kn[0] = t0 * Vj;
        kn[1] = t1 * Vj;
        kn[2] = t2 * Vj;
      } else {
        T4[slot] = Quad<TS>{{(TS)t0, (TS)t1, (TS)t2, (TS)0}};
      }
    } else {
      const double wj = Vj * iVh;
#pragma unroll
      for (int q = 0; q < 9; ++q) kn[q] = (Acc)(wj * SK[q]);
    }
    // point history: volume-weighted mean of the bond states
#pragma unroll
    for (int k = 0; k < 6; ++k) hs[k] += Vj * sgb[k];
    hpc += Vj * pcb;
    hw += Vj;
  };
  if (tid < nf) tail(tid);
  if (nf > kBondThreads) {                        // uniform per block
    double u[8];
    int ui[5];
    auto fold = [&](bool first) {
#pragma unroll
      for (int k = 0; k < 6; ++k) u[k] = (first ? 0.0 : u[k]) + wave_sum(hs[k]);
      u[6] = (first ? 0.0 : u[6]) + wave_sum(hpc);
      u[7] = (first ? 0.0 : u[7]) + wave_sum(hw);
      ui[0] = (first ? 0 : ui[0]) + wave_sum_i(n_deg);
      ui[1] = (first ? 0 : ui[1]) + wave_sum_i(n_pl);
      ui[2] = (first ? 0 : ui[2]) + wave_sum_i(n_nc);
      ui[3] = (first ? 0 : ui[3]) + wave_sum_i(n_trip);
      ui[4] = max(first ? 0 : ui[4], wave_max_i(mx));
#pragma unroll
      for (int k = 0; k < 6; ++k) hs[k] = 0.0;
      hpc = hw = 0.0;
      n_deg = n_pl = n_nc = n_trip = mx = 0;
    };
    fold(true);
    for (int m0 = kBondThreads; m0 < nf; m0 += kBondThreads) {   // uniform trip count:
      if (m0 + tid < nf) tail(m0 + tid);                          // the wave sums need
      fold(false);                                                // every lane
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) hs[k] = u[k];
      hpc = u[6]; hw = u[7];
      n_deg = ui[0]; n_pl = ui[1]; n_nc = ui[2]; n_trip = ui[3]; mx = ui[4];
    }
  }
  double own[3] = {0.0, 0.0, 0.0};
  if constexpr (kF64) if (P.force_mode == ULPPM_FORCE_EQ51 && A.fown) {
    // rows of the lane's own bonds (a degenerate bond's row reads zero)
    for (int m = tid; m < nf; m += kBondThreads) {
      own[0] += sKN[16 * (size_t)m];
      own[1] += sKN[16 * (size_t)m + 1];
      own[2] += sKN[16 * (size_t)m + 2];
    }
  }
  if constexpr (kF64) if (P.force_mode == ULPPM_FORCE_CONJUGATE) {
    // ---- pass 2 in FP64 on the VALU: A_k = sum_j B_kj M_j, streaming the
    // rows M_j of the (symmetric) membership matrix in groups of four.  FP64
    // matrix products run at the vector rate on this chip and would pad the
    // 9 outputs to 16.  Rows past the family up to a whole group read as
    // zeros (their membership bits are clear, and 0 * stale data could be NaN).
    // With the own sums kept here, the records hold V_i T_ik: the gather of
    // point k then needs no V_i of its neighbours.
    const double sc = A.fown ? A.vol_n[i] : 1.0;
    for (int m = nf + tid; m < 4 * nks; m += kBondThreads) {
#pragma unroll
      for (int q = 0; q < 9; ++q) sKN[16 * (size_t)m + q] = (Acc)0;
    }
    __syncthreads();
    if (kBondWaves == 2 && nf <= 2 * kWave && 16 * bond_mx_rows(mf) >= 18 * kWave) {
      // Two members per lane (k = lane and lane + 64), the groups of rows
      // split between the two waves: each row read from LDS serves two
      // members, which halves the LDS traffic that bounds this loop.  The
      // waves then hand each other the partial sums of the member the other
      // one finishes.
      const int gh = (nks + 1) / 2;
      const int g0 = wid == 0 ? 0 : gh, g1 = wid == 0 ? gh : nks;
      const int ka = lane, kb = lane + kWave;
      const bool va = ka < nf, vb = kb < nf;
      Acc Pa[9], Pb[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) Pa[t] = Pb[t] = (Acc)0;
      unsigned long long wa = 0ull, wb = 0ull;
      for (int g = g0; g < g1; ++g) {
        const int s4 = g & 15;
        if (g == g0 || s4 == 0) {                  // membership words of both members
          const unsigned long long xa = sb[(size_t)(va ? ka : 0) * nw + (g >> 4)];
          const unsigned long long xb = sb[(size_t)(vb ? kb : 0) * nw + (g >> 4)];
          wa = va ? xa : 0ull;
          wb = vb ? xb : 0ull;
        }
        Acc r[4][9];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const Acc* rq = sKN + 16 * (size_t)(4 * g + q);
#pragma unroll
          for (int t = 0; t < 9; ++t) r[q][t] = rq[t];
        }
        // members 4 g + q; their bits are 16 q + s4 of the word
        const unsigned la = (unsigned)wa, ha = (unsigned)(wa >> 32);
        const unsigned lb = (unsigned)wb, hb = (unsigned)(wb >> 32);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int sh = 16 * (q & 1) + s4;
          const Acc w0 = (Acc)(((q < 2 ? la : ha) >> sh) & 1u);
          const Acc w1 = (Acc)(((q < 2 ? lb : hb) >> sh) & 1u);
#pragma unroll
          for (int t = 0; t < 9; ++t) {
            Pa[t] += w0 * r[q][t];
            Pb[t] += w1 * r[q][t];
          }
        }
      }
      __syncthreads();                             // every row M_j has been read
      Acc* xch = sKN;                              // [18][64]: the partials handed over
      if (wid == 0) {
#pragma unroll
        for (int t = 0; t < 9; ++t) xch[(size_t)(9 + t) * kWave + lane] = Pb[t];
      } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) xch[(size_t)t * kWave + lane] = Pa[t];
      }
      __syncthreads();
      Acc S[9];
      if (wid == 0) {
#pragma unroll
        for (int t = 0; t < 9; ++t) S[t] = Pa[t] + xch[(size_t)t * kWave + lane];
      } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) S[t] = Pb[t] + xch[(size_t)(9 + t) * kWave + lane];
      }
      const int m = wid == 0 ? ka : kb;
      if (m < nf) {
        const Acc* zm = sR + 8 * (size_t)m;
        const Acc zx = zm[0] - xi0, zy = zm[1] - xi1, zz = zm[2] - xi2;
        const Acc t0 = S[0] * zx + S[1] * zy + S[2] * zz, t1 = S[3] * zx + S[4] * zy + S[5] * zz,
                  t2 = S[6] * zx + S[7] * zy + S[8] * zz;
        T4[b0 + m] = Quad<TS>{{(TS)(sc * t0), (TS)(sc * t1), (TS)(sc * t2), (TS)0}};
        own[0] += t0 * zm[3];                                      // sum_k T_ik V_k
        own[1] += t1 * zm[3];
        own[2] += t2 * zm[3];
      }
    } else {
      // one lane per member k (families of more than 128 members)
      for (int m = tid; m < nf; m += kBondThreads) {
        Acc a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0, a7 = 0, a8 = 0;
        for (int c = 0; c < nblk; ++c) {
          const unsigned long long word = sb[(size_t)m * nw + c];
          const unsigned lo = (unsigned)word, hi = (unsigned)(word >> 32);
          // members 64 c + 4 s + q in order; their bits are 16 q + s of the word
          for (int s4 = 0; s4 < 16; ++s4) {
            const int j0 = 64 * c + 4 * s4;
            if (j0 >= nf) break;
            Acc r[4][9];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const Acc* rq = sKN + 16 * (size_t)(j0 + q);
#pragma unroll
              for (int t = 0; t < 9; ++t) r[q][t] = rq[t];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const unsigned half = q < 2 ? lo : hi;
              const Acc w = (Acc)((half >> (16 * (q & 1) + s4)) & 1u);
              a0 += w * r[q][0]; a1 += w * r[q][1]; a2 += w * r[q][2];
              a3 += w * r[q][3]; a4 += w * r[q][4]; a5 += w * r[q][5];
              a6 += w * r[q][6]; a7 += w * r[q][7]; a8 += w * r[q][8];
            }
          }
        }
        const Acc* zm = sR + 8 * (size_t)m;
        const Acc zx = zm[0] - xi0, zy = zm[1] - xi1, zz = zm[2] - xi2;
        const int64_t slot = b0 + m;
        const Acc t0 = a0 * zx + a1 * zy + a2 * zz, t1 = a3 * zx + a4 * zy + a5 * zz, t2 = a6 * zx + a7 * zy + a8 * zz;
        T4[slot] = Quad<TS>{{(TS)(sc * t0), (TS)(sc * t1), (TS)(sc * t2), (TS)0}};
        own[0] += t0 * zm[3];                                      // sum_k T_ik V_k
        own[1] += t1 * zm[3];
        own[2] += t2 * zm[3];
      }
    }
  }
  if constexpr (!kF64) if (P.force_mode == ULPPM_FORCE_CONJUGATE) {
    // ---- pass 2 in FP32: A_k = sum_j B_kj M_j on the matrix cores
    // (membership is symmetric, so row k of the bit matrix is column k),
    // then T_ik = A_k zeta_ik with the three products of a row combined
    // across neighbouring lanes.
    __syncthreads();
    auto tiles2 = [&](int t0, auto nbc) {
      constexpr int NB = decltype(nbc)::value;
      V4 acc[NB];
      unsigned piece[NB];
      int krow[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        acc[b] = V4{0, 0, 0, 0};
        piece[b] = 0u;
        krow[b] = (t0 + kBondWaves * b) * 16 + r16;
      }
      for (int js = 0; js < nks; ++js) {
        const int j = 4 * js + q4;
        const bool ok = j < nf && r16 < 9;
        const Acc mv = sKN[16 * (size_t)(ok ? j : 0) + (r16 < 9 ? r16 : 0)];
        const Acc bval = ok ? mv : (Acc)0;
        const int s = js & 15;
        if (s == 0) {
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const bool kv = krow[b] < nf;
            const unsigned pw = sq[((size_t)(kv ? krow[b] : 0) * nw + (js >> 4)) * 4 + q4];
            piece[b] = kv ? pw : 0u;
          }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const Acc av = (piece[b] >> s) & 1u ? (Acc)1 : (Acc)0;
          acc[b] = MM::run(av, bval, acc[b]);
        }
      }
      const int qz = r16 % 3;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int t = t0 + kBondWaves * b;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = t * 16 + MM::row(q4, r);
          const bool ok = k < nf && r16 < 9;
          const Acc zq = sR[8 * (size_t)(ok ? k : 0) + qz];
          const Acc prod = ok ? acc[b][r] * zq : (Acc)0;
          const Acc p1 = __shfl_down(prod, 1, 16);
          const Acc p2 = __shfl_down(prod, 2, 16);
          if (ok && qz == 0) T4[b0 + k].v[r16 / 3] = (TS)(prod + p1 + p2);
        }
      }
    };
    for (int t0 = wid; t0 < ntile; t0 += kBondWaves * kTileBatch) {
      const int nb = (ntile - t0 + kBondWaves - 1) / kBondWaves;
      tile_slots(nb, t0, tiles2);
    }
  }
  mx = wave_max_i(mx);
  // Closing: the point-history sums, the own force-state sums and the
  // counters (15 rows of one double per thread) go through LDS.  Each row is
  // added by kLpr lanes, 16 entries each, then by DPP within the lanes; with
  // two waves, wave 0 holds rows 0-7 and writes the point history, wave 1
  // rows 8-14 and writes the own sums and counters.
  __syncthreads();   // the family's working set is no longer read
  constexpr int kLpr = kBondThreads / 16, kRpw = kWave / kLpr;   // lanes per row, rows per wave
  double* hred = reinterpret_cast<double*>(smem_raw);              // [16][kBondThreads]
  int* redm = reinterpret_cast<int*>(hred + 16 * kBondThreads);    // [waves]: max Newton iterations
  {
    const double rv[kCloseRows] = {hs[0], hs[1], hs[2], hs[3], hs[4], hs[5], hpc, hw, own[0], own[1], own[2],
                                   (double)n_deg, (double)n_pl, (double)n_nc, (double)n_trip};
#pragma unroll
    for (int k = 0; k < kCloseRows; ++k) hred[k * kBondThreads + tid] = rv[k];
    hred[kCloseRows * kBondThreads + tid] = 0.0;
  }
  if (lane == 0) redm[wid] = mx;
  __syncthreads();
  double v = 0.0;
  {
    const double* src = hred + (tid / kLpr) * kBondThreads + (tid % kLpr) * 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) v += src[e];
  }
  v += dpp_d<kDppXor1, 0xF>(v);
  v += dpp_d<kDppXor2, 0xF>(v);
  if constexpr (kLpr == 8) v += dpp_d<kDppHalfMirror, 0xF>(v);
  const long long vb = __double_as_longlong(v);
  double tot[kRpw];                                               // this wave's rows, uniform
#pragma unroll
  for (int k = 0; k < kRpw; ++k)
    tot[k] = __longlong_as_double(((long long)__builtin_amdgcn_readlane((int)(vb >> 32), k * kLpr) << 32) |
                                  (unsigned)__builtin_amdgcn_readlane((int)vb, k * kLpr));
  if (lane != 0) return;
  if (wid == 0) {                                                 // rows 0-7
    const double W = tot[7];
    if (W > 0.0) {
      for (int k = 0; k < 6; ++k) A.sig_out[k][i] = tot[k] / W;
      A.pc_out[i] = tot[6] / W;
    } else {
      for (int k = 0; k < 6; ++k) A.sig_out[k][i] = sig_i[k];
      A.pc_out[i] = pc_i;
    }
  }
  if (wid == 8 / kRpw) {                                          // rows 8-14
    const double* t = tot + (8 - wid * kRpw);
    if (A.fown)
      for (int c = 0; c < 3; ++c) A.fown[c * n + i] = t[c];
    const long long d = (long long)t[3], pl = (long long)t[4], nc = (long long)t[5], tr = (long long)t[6];
    int m2 = 0;
    for (int w = 0; w < kBondWaves; ++w) m2 = m2 > redm[w] ? m2 : redm[w];
    if (d) ctr_add(A.ctr, C_DEGEN, (unsigned long long)d);
    if (pl) ctr_add(A.ctr, C_PLASTIC, (unsigned long long)pl);
    if (nc) ctr_add(A.ctr, C_NOCONV, (unsigned long long)nc);
    ctr_add(A.ctr, C_TRIPLES, (unsigned long long)tr);
    ctr_add(A.ctr, C_TESTS, (unsigned long long)((long long)nf * nf));
    if (m2) ctr_max(A.ctr, C_MAXNEWTON, (unsigned long long)m2);
  }
}

// ------------------------------------------------------------- adjoint --
// Reverse mode of one step n -> n+1 with the step's sets frozen (families,
// sub-horizons, degenerate bonds, elastic/plastic branches).  The forward
// step is first re-run on a scratch copy of state n, which leaves x^{n+1},
// v_half, V^n, the families and the force states in the context.

// Partial derivatives of the retention curve (Eq. 15 as read) in J, phi, s.
__host__ __device__ void swrc_grad(const DevParams& P, double J, double phi, double s, double* dJ, double* dphi,
                                   double* ds) {
  *dJ = *dphi = *ds = 0.0;
  if (!(s > 0.0)) return;
  const double e = phi / (1.0 - phi);
  const double X = P.a1 * pow(e, P.a2) * J * (s * 1e-3);
  const double m = (P.n_vg - 1.0) / P.n_vg;
  const double Xn = pow(X, P.n_vg);
  const double dSdX = -m * pow(1.0 + Xn, -m - 1.0) * P.n_vg * Xn / X;
  *dJ = dSdX * X / J;
  *dphi = dSdX * X * P.a2 / (e * (1.0 - phi) * (1.0 - phi));
  *ds = dSdX * X / s;
}

struct AdjArgs {
  int64_t n, per;
  const int64_t* row;
  const int32_t* col;
  const int32_t* rev;
  const double* x;        // x^{n+1} (3n)
  const double* vh;       // v_half (3n)
  const double* vol_n;    // V^n
  const double* xv;       // 8n packed x^{n+1}, V^n, v_half
  const double* J;        // state n
  const double* phi;
  const double* s;
  const double* sig[6];
  const double* pc;
  const double* J1;       // state n+1
  const double* phi1;
  const double* Sr1;
  const double* V1;
  const double* sig1[6];
  const double* pc1;
  const double* fbar;     // 3n, adjoint of the nodal force
  const double* Mbt;      // n, adjoint of M^{n+1} including the acceleration term
  const double* Vb1;      // incoming adjoints of state n+1
  const double* phib1;
  const double* Jb1;
  const double* Srb1;
  const double* sigb1[6];
  const double* pcb1;
  double* own_x;          // 3n: -sum_k zeta_bar_ik
  double* own_vh;         // 3n: -sum_k ydot_bar_ik
  double* own_V;          // n
  double* sigb;           // 6n adjoint of sigma^n
  double* pcb;            // n
  double* Jb;             // n
  double* phib;           // n
  double* sb;             // n, this step's suction adjoint
  // One 64-byte record per bond slot (i,k), the contributions of point i to
  // the adjoints of point k: xbar_k (3), vhbar_k (3), Vbar_k (1), 0.  The
  // three pointers address its fields; the record of slot s starts at 8 s.
  double* slot_x;
  double* slot_vh;
  double* slot_V;
  double* fwd;            // 8 x cap: the bond tail's forward solution per slot (sigma 6, p_c, branch)
  double* thpart;         // 4 per block
  unsigned long long* ctr;  // striped counters (C_ADJLDS)
  // history on the bonds: start states of this step's bonds (8 per slot),
  // adjoints of their updated states (8 per slot), adjoints of the start
  // states (8 per slot, written)
  const double* hstart = nullptr;
  const double* hbar1 = nullptr;
  double* hbar0s = nullptr;
  int64_t cap;
  double dt;
  int max_f;
};

template <class T>
__host__ __device__ __forceinline__ void sym_full_grad(const double* Kb, double* Ks) {
  // symmetric matrix Ks = G + G^T from the unique-entry gradient Kb (Voigt)
  Ks[0] = 2.0 * Kb[0]; Ks[1] = 2.0 * Kb[1]; Ks[2] = 2.0 * Kb[2];
  Ks[3] = Kb[3]; Ks[4] = Kb[4]; Ks[5] = Kb[5];
}

__host__ __device__ __forceinline__ void symv(const double* S, const double* z, double* out) {
  out[0] = S[0] * z[0] + S[5] * z[1] + S[4] * z[2];
  out[1] = S[5] * z[0] + S[1] * z[1] + S[3] * z[2];
  out[2] = S[4] * z[0] + S[3] * z[1] + S[2] * z[2];
}

// Positions x^{n+1} = x0 + u^{n+1} from state n+1 and v_half, V^n from state
// n, exactly as the predictor formed them.
__global__ void k_adj_kin(ulppm_state S, ulppm_state S1, DevParams P, double* __restrict__ x,
                          double* __restrict__ vh, double* __restrict__ vol_n) {
#pragma clang fp contract(off)
  const int64_t n = S.n;
  const double hdt = 0.5 * P.dt;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const bool fx = S.fixed[i] != 0, drv = S.fixed[i] == 2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vh[c * n + i] = drv ? S.v[c][i] : fx ? 0.0 : S.v[c][i] + hdt * S.a[c][i];
      x[c * n + i] = S1.x0[c][i] + S1.u[c][i];
    }
    vol_n[i] = S.vol[i];
  }
}

__global__ __launch_bounds__(256) void k_adj_point1(int64_t n, const uint8_t* __restrict__ fixed,
                                                    const double* __restrict__ a1x, const double* __restrict__ a1y,
                                                    const double* __restrict__ a1z, const double* __restrict__ M1,
                                                    const double* __restrict__ vbx, const double* __restrict__ vby,
                                                    const double* __restrict__ vbz, const double* __restrict__ abx,
                                                    const double* __restrict__ aby, const double* __restrict__ abz,
                                                    const double* __restrict__ Mb1, double h, double g0, double g1,
                                                    double g2, double* __restrict__ fbar, double* __restrict__ Mbt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    // v' = v_half + h a', a' = f/M' + g (free points)
    const double at[3] = {abx[i] + h * vbx[i], aby[i] + h * vby[i], abz[i] + h * vbz[i]};
    double mb = Mb1[i];
    if (fixed[i]) {
      fbar[i] = fbar[n + i] = fbar[2 * n + i] = 0.0;
    } else {
      const double M = M1[i];
      const double a[3] = {a1x[i], a1y[i], a1z[i]}, g[3] = {g0, g1, g2};
      for (int c = 0; c < 3; ++c) {
        fbar[c * n + i] = at[c] / M;
        mb -= at[c] * (a[c] - g[c]) / M;    // f/M^2 = (a - g)/M
      }
    }
    Mbt[i] = mb;
  }
}

// One workgroup per point i: re-run the bond pass of i, then reverse it.
// The masked sums of the re-run pass 1 and of the reverse of the sums are
// membership-matrix products on the matrix cores (16x16x4 FP64, the lane
// layout of the forward bond kernel); the 9-column sums stay on the VALU.
// Hist: the history on the bonds; each bond starts from its carried state
// (A.hstart), its updated state also receives A.hbar1, and the adjoint of
// its start state goes to A.hbar0s instead of the point's history.
// LinP: the linear pre-consolidation law (b1 = 0, b2 = 1), as in the forward
// bond kernel.
template <bool Hist, class Acc, bool LinP>
__global__ __launch_bounds__(kBondThreads, ULPPM_ADJ_MIN_WAVES) void k_adj_bond(AdjArgs A, DevParams P) {
  using MM = Mma<Acc>;            // the two membership-matrix sweeps: FP64, or FP32 in mixed precision
  using V4 = typename MM::V;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t i = xcd_point(blockIdx.x, A.per);
  if (i >= A.n) {                                 // idle block: its parameter partials are zero
    if (threadIdx.x < 4) A.thpart[4 * blockIdx.x + threadIdx.x] = 0.0;
    return;
  }
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int mf = A.max_f;
  const int64_t n = A.n;
  const int64_t b0 = A.row[i];
  const int nf = (int)(A.row[i + 1] - b0);
  if (nf > mf) {                                  // the LDS was laid out for fewer members
    if (tid == 0) ctr_add(A.ctr, C_ADJLDS, 1ull);
    if (tid < 4) A.thpart[4 * blockIdx.x + tid] = 0.0;
    return;                                       // uniform per block; the step reports an error
  }
  const int nw = (mf + 63) / 64;
  // LDS per member: 3 quads, the 10-value record and the 16 sums (320 B with
  // two membership words), so that four workgroups fit a CU for families of
  // up to ~124.  The per-bond adjoint partials of zeta and V live in their
  // output slots (A.slot_x, A.slot_V) and the tail's forward solution in
  // A.fwd, both in HBM, read back by the thread that wrote them.
  Quad<double>* sX = reinterpret_cast<Quad<double>*>(smem_raw);   // x_k (pass 1), Tbar_ik, then H columns 10-13
  Quad<double>* sTb = sX;
  Quad<double>* sZ = sX + mf;                                     // zeta_ik, V_k
  Quad<double>* sY = sZ + mf;                                     // ydot_ik, 1 (then H column 14)
  MRec<double>* sM = reinterpret_cast<MRec<double>*>(sY + mf);    // M_j, then G and H columns 0-9
  double* sKN = reinterpret_cast<double*>(sM + mf);               // 16 per bond: K(6) N(9) active | Ks(6) Nb(9)
  unsigned long long* sb = reinterpret_cast<unsigned long long*>(sKN + 16 * (size_t)mf);
  unsigned short* sq = reinterpret_cast<unsigned short*>(sb);     // membership quarters, as the forward
  __shared__ double red[kBondWaves][32];
  __shared__ double pt[32];
  __shared__ double s_Pn;

  const double xi0 = A.x[i], xi1 = A.x[n + i], xi2 = A.x[2 * n + i];
  const double vi0 = A.vh[i], vi1 = A.vh[n + i], vi2 = A.vh[2 * n + i];
  const double Vi = A.vol_n[i];
  const double fb_i[3] = {A.fbar[i], A.fbar[n + i], A.fbar[2 * n + i]};

  // ---- stage the family and the full-horizon sums (as the forward)
  double Kp[6] = {0, 0, 0, 0, 0, 0}, Np[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Vp = 0.0;
  for (int m = tid; m < nf; m += kBondThreads) {
    const int32_t k = A.col[b0 + m];
    const double4 pa = reinterpret_cast<const double4*>(A.xv)[2 * (int64_t)k];
    const double4 pb = reinterpret_cast<const double4*>(A.xv)[2 * (int64_t)k + 1];
    const double xk0 = pa.x, xk1 = pa.y, xk2 = pa.z, V = pa.w;
    const double z0 = xk0 - xi0, z1 = xk1 - xi1, z2 = xk2 - xi2;
    const double y0 = pb.x - vi0, y1 = pb.y - vi1, y2 = pb.z - vi2;
    sX[m] = Quad<double>{{xk0, xk1, xk2, V}};
    sZ[m] = Quad<double>{{z0, z1, z2, V}};
    sY[m] = Quad<double>{{y0, y1, y2, 1.0}};
    const double w0 = V * z0, w1 = V * z1, w2 = V * z2;
    Kp[0] += w0 * z0; Kp[1] += w1 * z1; Kp[2] += w2 * z2;
    Kp[3] += w1 * z2; Kp[4] += w0 * z2; Kp[5] += w0 * z1;
    Np[0] += y0 * w0; Np[1] += y0 * w1; Np[2] += y0 * w2;
    Np[3] += y1 * w0; Np[4] += y1 * w1; Np[5] += y1 * w2;
    Np[6] += y2 * w0; Np[7] += y2 * w1; Np[8] += y2 * w2;
    Vp += V;
  }
  for (int k = 0; k < 6; ++k) Kp[k] = wave_sum(Kp[k]);
  for (int k = 0; k < 9; ++k) Np[k] = wave_sum(Np[k]);
  Vp = wave_sum(Vp);
  if (lane == 0) {
    for (int k = 0; k < 6; ++k) red[wid][k] = Kp[k];
    for (int k = 0; k < 9; ++k) red[wid][6 + k] = Np[k];
    red[wid][15] = Vp;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 0; k < 16; ++k) {
      double a = 0.0;
      for (int w = 0; w < kBondWaves; ++w) a += red[w][k];
      pt[k] = a;                                   // K_i (6), N_i (9), Vh
    }
  }
  if (tid == kWave) s_Pn = apparent_pc<LinP>(P, A.pc[i]);   // Eq. 45, shared by the bonds of i
  __syncthreads();
  const double Vh = pt[15];
  const double Sr1 = A.Sr1[i], s_i = A.s[i];
  const double Srs = Sr1 * s_i;
  double sig_i[6];
  for (int k = 0; k < 6; ++k) sig_i[k] = A.sig[k][i];
  const double pc_i = A.pc[i];
  const double d2 = P.d2;
  const double dt = A.dt;

  const double Pn_i = s_Pn;
  const int ntile = (nf + 15) >> 4;
  const int nks = (nf + 3) >> 2;

  // ---- pass 1 (re-run): [K_j | N_j | count] = B [V zeta zeta^T | V ydot zeta^T | 1]
  {
    // feature f of member k is V a b from {zeta0, zeta1, zeta2, V, ydot0, ydot1, ydot2, 1}
    // (sZ and sY are adjacent); feature 15 counts the members
    const int fa = feat_a(r16), fb = feat_b(r16), fv = r16 == 15 ? 7 : 3;
    const double* rz = &sZ[0].v[0];
    const int oa = fa < 4 ? fa : 4 * mf + fa - 4, ob = fb < 4 ? fb : 4 * mf + fb - 4,
              ov = fv < 4 ? fv : 4 * mf + fv - 4;
    auto tiles = [&](int t0, auto nbc) {
      constexpr int NB = decltype(nbc)::value;
      double xj[NB][3];
      bool jv[NB];
      int jrow[NB];
      V4 acc[NB];
      unsigned piece[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        jrow[b] = (t0 + kBondWaves * b) * 16 + r16;
        jv[b] = jrow[b] < nf;
        const Quad<double> q = sX[jv[b] ? jrow[b] : 0];     // positions: the test of Eq. 22
        xj[b][0] = q.v[0]; xj[b][1] = q.v[1]; xj[b][2] = q.v[2];
        acc[b] = V4{0, 0, 0, 0};
        piece[b] = 0u;
      }
      for (int ks = 0; ks < nks; ++ks) {
        const int kk0 = 4 * ks + q4;
        const bool kv = kk0 < nf;
        const int kk = kv ? kk0 : 0;
        const Quad<double> xk = sX[kk];
        const double fvv = rz[4 * kk + oa] * rz[4 * kk + ob] * rz[4 * kk + ov];
        const Acc bval = kv ? (Acc)fvv : (Acc)0;
        const unsigned sbit = 1u << (ks & 15);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const bool in = within(xj[b][0], xj[b][1], xj[b][2], xk.v[0], xk.v[1], xk.v[2], d2) & kv & jv[b];
          piece[b] |= in ? sbit : 0u;
          acc[b] = MM::run(in ? (Acc)1 : (Acc)0, bval, acc[b]);
        }
        if ((ks & 15) == 15 || ks == nks - 1) {
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            if (jv[b]) sq[((size_t)jrow[b] * nw + (ks >> 4)) * 4 + q4] = (unsigned short)piece[b];
            piece[b] = 0u;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int t = t0 + kBondWaves * b;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = t * 16 + MM::row(q4, r);
          if (j < nf) sKN[16 * (size_t)j + r16] = acc[b][r];
        }
      }
    };
    for (int t0 = wid; t0 < ntile; t0 += kBondWaves * kTileBatch) {
      const int nb = (ntile - t0 + kBondWaves - 1) / kBondWaves;     // slots left for this wave
      tile_slots(nb, t0, tiles);
    }
  }
  __syncthreads();

  // ---- tail forward, one lane per bond
  double Wp = 0.0;
  for (int m = tid; m < nf; m += kBondThreads) {
    double* kn = sKN + 16 * (size_t)m;
    double Kq[6], Nq[9];
    for (int k = 0; k < 6; ++k) Kq[k] = kn[k];
    for (int k = 0; k < 9; ++k) Nq[k] = kn[6 + k];
    const int ns = (int)kn[15];
    const bool active = shape_regular(P.plane != 0, Kq, ns);
    kn[15] = active ? 1.0 : 0.0;
    MRec<double> r{};
    if (active) {
      const double Vj = sZ[m].v[3];
      TailFwd F;
      if constexpr (Hist) {
        const double* h0 = A.hstart + 8 * (b0 + m);
        tail_forward_pn<LinP>(P, Kq, Nq, h0, h0[6], apparent_pc<LinP>(P, h0[6]), Srs, Vj / Vh, dt, F);
      } else {
        tail_forward_pn<LinP>(P, Kq, Nq, sig_i, pc_i, Pn_i, Srs, Vj / Vh, dt, F);
      }
      for (int q = 0; q < 9; ++q) r.v[q] = F.M[q];
      double* rr = A.fwd + 8 * (b0 + m);
      for (int k = 0; k < 6; ++k) rr[k] = F.sg[k];
      rr[6] = F.pc;
      rr[7] = (double)F.branch;
      Wp += Vj;
    }
    sM[m] = r;
  }
  Wp = wave_sum(Wp);
  if (lane == 0) red[wid][16] = Wp;
  __syncthreads();
  double W = 0.0;
  for (int w = 0; w < kBondWaves; ++w) W += red[w][16];

  // ---- pass 2 (re-run) and the reverse of the gather:
  // Tbar_ik = V_i V_k (fbar_i - fbar_k); zeta_bar_ik = A_ik^T Tbar_ik with
  // A_ik = sum_j B_kj M_j; volume adjoints of the gather.
  double ownV = 0.0;
  // the reverse of the gather for member m, given A_ik
  auto gather_reverse = [&](int m, const double* a) {
    const int64_t slot = b0 + m;
    const int32_t k = A.col[slot];
    const double Vk = sZ[m].v[3];
    const double fb_k[3] = {A.fbar[k], A.fbar[n + k], A.fbar[2 * n + k]};
    const double df[3] = {fb_i[0] - fb_k[0], fb_i[1] - fb_k[1], fb_i[2] - fb_k[2]};
    double tb[3];
    for (int c = 0; c < 3; ++c) tb[c] = Vi * Vk * df[c];
    sTb[m] = Quad<double>{{tb[0], tb[1], tb[2], 0.0}};
    Quad<double> zb;
    zb.v[0] = a[0] * tb[0] + a[3] * tb[1] + a[6] * tb[2];
    zb.v[1] = a[1] * tb[0] + a[4] * tb[1] + a[7] * tb[2];
    zb.v[2] = a[2] * tb[0] + a[5] * tb[1] + a[8] * tb[2];
    // With symmetric families, sum_i fbar_i . f_i = sum_i sum_k V_i V_k
    // T_ik . (fbar_i - fbar_k): the volume adjoints need only this point's
    // own force states T_ik = A_ik zeta_ik.
    const Quad<double> zq = sZ[m];
    double e = 0.0;
    for (int c = 0; c < 3; ++c) e += (a[3 * c] * zq.v[0] + a[3 * c + 1] * zq.v[1] + a[3 * c + 2] * zq.v[2]) * df[c];
    ownV += Vk * e;
    zb.v[3] = Vi * e;                               // to Vbar_k
    for (int c = 0; c < 3; ++c) A.slot_x[8 * slot + c] = zb.v[c];
    A.slot_V[8 * slot] = zb.v[3];
  };
  if (kBondWaves == 2 && nf <= 2 * kWave && (size_t)mf * sizeof(MRec<double>) >= 18 * kWave * sizeof(double)) {
    // Two members per lane (k = lane and lane + 64), the groups of rows split
    // between the waves, which then hand each other the partial sums of the
    // member the other finishes (as the forward pass 2).  Rows past the family
    // are clamped and enter with weight 0.
    const int gh = (nks + 1) / 2;
    const int g0 = wid == 0 ? 0 : gh, g1 = wid == 0 ? gh : nks;
    const int ka = lane, kb = lane + kWave;
    const bool va = ka < nf, vb = kb < nf;
    double Pa[9], Pb[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Pa[e] = Pb[e] = 0.0;
    unsigned long long wa = 0ull, wb = 0ull;
    for (int g = g0; g < g1; ++g) {
      const int s4 = g & 15, j0 = 4 * g;
      if (g == g0 || s4 == 0) {
        const unsigned long long xa = sb[(size_t)(va ? ka : 0) * nw + (g >> 4)];
        const unsigned long long xb = sb[(size_t)(vb ? kb : 0) * nw + (g >> 4)];
        wa = va ? xa : 0ull;
        wb = vb ? xb : 0ull;
      }
      MRec<double> r4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) r4[q] = sM[j0 + q < nf ? j0 + q : nf - 1];
      const unsigned la = (unsigned)wa, ha = (unsigned)(wa >> 32);
      const unsigned lb = (unsigned)wb, hb = (unsigned)(wb >> 32);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int sh = 16 * (q & 1) + s4;
        const double w0 = (double)(((q < 2 ? la : ha) >> sh) & 1u);
        const double w1 = (double)(((q < 2 ? lb : hb) >> sh) & 1u);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
          Pa[e] += w0 * r4[q].v[e];
          Pb[e] += w1 * r4[q].v[e];
        }
      }
    }
    __syncthreads();                               // every row M_j has been read
    double* xch = reinterpret_cast<double*>(sM);   // [18][64]; sM is free until the G/H sweep
    if (wid == 0) {
#pragma unroll
      for (int e = 0; e < 9; ++e) xch[(size_t)(9 + e) * kWave + lane] = Pb[e];
    } else {
#pragma unroll
      for (int e = 0; e < 9; ++e) xch[(size_t)e * kWave + lane] = Pa[e];
    }
    __syncthreads();
    double a[9];
    if (wid == 0) {
#pragma unroll
      for (int e = 0; e < 9; ++e) a[e] = Pa[e] + xch[(size_t)e * kWave + lane];
    } else {
#pragma unroll
      for (int e = 0; e < 9; ++e) a[e] = Pb[e] + xch[(size_t)(9 + e) * kWave + lane];
    }
    const int m = wid == 0 ? ka : kb;
    if (m < nf) gather_reverse(m, a);
  } else {
    for (int m = tid; m < nf; m += kBondThreads) {
      double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      // members 64 c + 4 s + q in groups of four (bits 16 q + s of word c);
      // rows past the family are clamped and enter with weight 0
      for (int c = 0; 64 * c < nf; ++c) {
        const unsigned long long word = sb[(size_t)m * nw + c];
        const unsigned lo = (unsigned)word, hi = (unsigned)(word >> 32);
        for (int s4 = 0; s4 < 16; ++s4) {
          const int j0 = 64 * c + 4 * s4;
          if (j0 >= nf) break;
          MRec<double> r4[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) r4[q] = sM[j0 + q < nf ? j0 + q : nf - 1];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double w = (double)(((q < 2 ? lo : hi) >> (16 * (q & 1) + s4)) & 1u);
#pragma unroll
            for (int e = 0; e < 9; ++e) a[e] += w * r4[q].v[e];
          }
        }
      }
      gather_reverse(m, a);
    }
  }
  __syncthreads();

  // ---- Mbar_j = sum_k B_jk Tbar_ik zeta_ik^T for every bond, before the
  // tail: two members per lane with the groups split between the waves, as
  // above; the sums land in sM (free until the G/H sweep) for the tail.
  const bool mbar_swept = kBondWaves == 2 && nf <= 2 * kWave &&
                          (size_t)mf * sizeof(MRec<double>) >= 18 * kWave * sizeof(double);
  if (mbar_swept) {
    const int gh = (nks + 1) / 2;
    const int g0 = wid == 0 ? 0 : gh, g1 = wid == 0 ? gh : nks;
    const int ka = lane, kb = lane + kWave;
    const bool va = ka < nf, vb = kb < nf;
    double Pa[9], Pb[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Pa[e] = Pb[e] = 0.0;
    unsigned long long wa = 0ull, wb = 0ull;
    for (int g = g0; g < g1; ++g) {
      const int s4 = g & 15, t0 = 4 * g;
      if (g == g0 || s4 == 0) {
        const unsigned long long xa = sb[(size_t)(va ? ka : 0) * nw + (g >> 4)];
        const unsigned long long xb = sb[(size_t)(vb ? kb : 0) * nw + (g >> 4)];
        wa = va ? xa : 0ull;
        wb = vb ? xb : 0ull;
      }
      Quad<double> tb4[4], z4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = t0 + q < nf ? t0 + q : nf - 1;
        tb4[q] = sTb[t];
        z4[q] = sZ[t];
      }
      const unsigned la = (unsigned)wa, ha = (unsigned)(wa >> 32);
      const unsigned lb = (unsigned)wb, hb = (unsigned)(wb >> 32);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int sh = 16 * (q & 1) + s4;
        const double w0 = (double)(((q < 2 ? la : ha) >> sh) & 1u);
        const double w1 = (double)(((q < 2 ? lb : hb) >> sh) & 1u);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const double t0a = w0 * tb4[q].v[r], t0b = w1 * tb4[q].v[r];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Pa[3 * r + c] += t0a * z4[q].v[c];
            Pb[3 * r + c] += t0b * z4[q].v[c];
          }
        }
      }
    }
    __syncthreads();                               // sM is free: M_j was last read by the A_k sweep
    double* xch = reinterpret_cast<double*>(sM);   // [18][64]
    if (wid == 0) {
#pragma unroll
      for (int e = 0; e < 9; ++e) xch[(size_t)(9 + e) * kWave + lane] = Pb[e];
    } else {
#pragma unroll
      for (int e = 0; e < 9; ++e) xch[(size_t)e * kWave + lane] = Pa[e];
    }
    __syncthreads();
    double mbs[9];
    if (wid == 0) {
#pragma unroll
      for (int e = 0; e < 9; ++e) mbs[e] = Pa[e] + xch[(size_t)e * kWave + lane];
    } else {
#pragma unroll
      for (int e = 0; e < 9; ++e) mbs[e] = Pb[e] + xch[(size_t)(9 + e) * kWave + lane];
    }
    __syncthreads();
    const int m = wid == 0 ? ka : kb;
    if (m < nf) {
      MRec<double> r;
#pragma unroll
      for (int e = 0; e < 9; ++e) r.v[e] = mbs[e];
      r.v[9] = 0.0;
      sM[m] = r;
    }
    __syncthreads();
  }

  // ---- reverse of the force states (R5) and of the bond tail
  const double sgb1[6] = {A.sigb1[0][i], A.sigb1[1][i], A.sigb1[2][i], A.sigb1[3][i], A.sigb1[4][i], A.sigb1[5][i]};
  const double pcb1 = A.pcb1[i];
  double sig1[6];
  for (int k = 0; k < 6; ++k) sig1[k] = A.sig1[k][i];
  const double pc1 = A.pc1[i];
  double acc_sig[6] = {0, 0, 0, 0, 0, 0}, acc_pc = 0.0, acc_Srs = 0.0, acc_Vh = 0.0, acc_th[4] = {0, 0, 0, 0};
  // One lane per bond, the first bond of each lane with its sums starting at
  // zero (none carried through the reverse of its return map); further bonds
  // of a family wider than the workgroup carry them as wave totals.
  auto rtail = [&](const int m) {
    double* kn = sKN + 16 * (size_t)m;
    const bool active = kn[15] != 0.0;
    double Kb[6] = {0, 0, 0, 0, 0, 0}, Nb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (active) {
      // Mbar_j = sum_k B_jk Tbar_ik zeta_ik^T (swept above, or here one bond per lane)
      double mb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      if (mbar_swept) {
        const MRec<double> r = sM[m];
#pragma unroll
        for (int e = 0; e < 9; ++e) mb[e] = r.v[e];
      }
      for (int c = 0; !mbar_swept && 64 * c < nf; ++c) {   // members in groups of four, as above
        const unsigned long long word = sb[(size_t)m * nw + c];
        const unsigned lo = (unsigned)word, hi = (unsigned)(word >> 32);
        for (int s4 = 0; s4 < 16; ++s4) {
          const int t0 = 64 * c + 4 * s4;
          if (t0 >= nf) break;
          Quad<double> tb4[4], z4[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int t = t0 + q < nf ? t0 + q : nf - 1;
            tb4[q] = sTb[t];
            z4[q] = sZ[t];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double w = (double)(((q < 2 ? lo : hi) >> (16 * (q & 1) + s4)) & 1u);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
              const double wt = w * tb4[q].v[r];
              mb[3 * r] += wt * z4[q].v[0];
              mb[3 * r + 1] += wt * z4[q].v[1];
              mb[3 * r + 2] += wt * z4[q].v[2];
            }
          }
        }
      }
      double Kq[6], Nq[9];
      for (int k = 0; k < 6; ++k) Kq[k] = kn[k];
      for (int k = 0; k < 9; ++k) Nq[k] = kn[6 + k];
      const double Vj = sZ[m].v[3];
      TailFwd F;                                   // the return map's solution from pass 1
      tail_kinematics(P.plane != 0, Kq, Nq, dt, F);
      const double* rr = A.fwd + 8 * (b0 + m);
      for (int k = 0; k < 6; ++k) F.sg[k] = rr[k];
      F.pc = rr[6];
      F.branch = (int)rr[7];
      // history: sigma'_i = sum_j V_j sigma_ij / W
      double sgx[6];
      double vh_hist = 0.0;
      for (int k = 0; k < 6; ++k) {
        sgx[k] = sgb1[k] * Vj / W;
        vh_hist += sgb1[k] * (F.sg[k] - sig1[k]);
      }
      vh_hist += pcb1 * (F.pc - pc1);
      double pcx = pcb1 * Vj / W;
      double wb = 0.0;
      if constexpr (Hist) {
        // the bond's own updated state is also carried to the next step
        const double* hb = A.hbar1 + 8 * (b0 + m);
        for (int k = 0; k < 6; ++k) sgx[k] += hb[k];
        pcx += hb[6];
        const double* h0 = A.hstart + 8 * (b0 + m);
        double s0b[6] = {0, 0, 0, 0, 0, 0}, p0b = 0.0;
        tail_reverse<LinP>(P, Kq, Nq, h0, h0[6], Srs, Vj / Vh, dt, F, mb, sgx, pcx, Kb, Nb, s0b, &p0b, &acc_Srs,
                     &wb, acc_th);
        double* ho = A.hbar0s + 8 * (b0 + m);
        for (int k = 0; k < 6; ++k) ho[k] = s0b[k];
        ho[6] = p0b;
        ho[7] = 0.0;
      } else {
        tail_reverse<LinP>(P, Kq, Nq, sig_i, pc_i, Srs, Vj / Vh, dt, F, mb, sgx, pcx, Kb, Nb, acc_sig, &acc_pc,
                     &acc_Srs, &wb, acc_th);
      }
      // w_j = V_j / Vh
      A.slot_V[8 * (b0 + m)] += wb / Vh + vh_hist / W;
      acc_Vh -= wb * Vj / (Vh * Vh);
    }
    if constexpr (Hist) {
      if (!active) {                               // an inactive bond keeps its start state
        const double* hb = A.hbar1 + 8 * (b0 + m);
        double* ho = A.hbar0s + 8 * (b0 + m);
        for (int k = 0; k < 8; ++k) ho[k] = hb[k];
      }
    }
    double Ks[6];
    sym_full_grad<double>(Kb, Ks);
    for (int k = 0; k < 6; ++k) kn[k] = Ks[k];
    for (int k = 0; k < 9; ++k) kn[6 + k] = Nb[k];
  };
  if (tid < nf) rtail(tid);
  if (nf > kBondThreads) {                        // uniform per block
    double u[13];
    auto fold = [&](bool first) {
      double* acc[13] = {&acc_sig[0], &acc_sig[1], &acc_sig[2], &acc_sig[3], &acc_sig[4], &acc_sig[5], &acc_pc,
                         &acc_Srs, &acc_Vh, &acc_th[0], &acc_th[1], &acc_th[2], &acc_th[3]};
#pragma unroll
      for (int k = 0; k < 13; ++k) {
        u[k] = (first ? 0.0 : u[k]) + wave_sum(*acc[k]);
        *acc[k] = 0.0;
      }
    };
    fold(true);
    for (int m0 = kBondThreads; m0 < nf; m0 += kBondThreads) {   // uniform trip count
      if (m0 + tid < nf) rtail(m0 + tid);
      fold(false);
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) acc_sig[k] = u[k];
      acc_pc = u[6]; acc_Srs = u[7]; acc_Vh = u[8];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc_th[k] = u[9 + k];
    }
  }
  // block reductions: sigma_bar_i (6), pc_bar_i, Srs_bar, Vh_bar, theta (4), own V (gather)
  double vals[14] = {acc_sig[0], acc_sig[1], acc_sig[2], acc_sig[3], acc_sig[4], acc_sig[5], acc_pc, acc_Srs,
                     acc_Vh, acc_th[0], acc_th[1], acc_th[2], acc_th[3], ownV};
  for (int k = 0; k < 14; ++k) vals[k] = wave_sum(vals[k]);
  __syncthreads();
  if (lane == 0)
    for (int k = 0; k < 14; ++k) red[wid][k] = vals[k];
  __syncthreads();
  if (tid == 0) {
    double v[14];
    for (int k = 0; k < 14; ++k) {
      v[k] = 0.0;
      for (int w = 0; w < kBondWaves; ++w) v[k] += red[w][k];
    }
    double Vb_own = v[13];                       // gather: sum_k V_k (T_ik - T_ki).fbar_i
    // history with no active bond keeps the point state
    if (!(W > 0.0)) {
      for (int k = 0; k < 6; ++k) v[k] += sgb1[k];
      v[6] += pcb1;
    }
    for (int k = 0; k < 6; ++k) A.sigb[k * n + i] = v[k];
    A.pcb[i] = v[6];
    const double Srsb = v[7];
    double Vhb = v[8];
    for (int k = 0; k < 4; ++k) A.thpart[4 * blockIdx.x + k] = v[9 + k];
    // point kinematics reverse (Eqs. 15-17, 48)
    const double J0 = A.J[i], phi0 = A.phi[i], V0 = Vi;
    const double J1 = A.J1[i], phi1 = A.phi1[i], V1 = A.V1[i];
    const double Jd = V1 / V0;
    const double Mb = A.Mbt[i];
    double V1b = A.Vb1[i] + Mb * (P.rho_s * (1.0 - phi1) + P.rho_w * Sr1 * phi1);
    double phi1b = A.phib1[i] + Mb * V1 * (P.rho_w * Sr1 - P.rho_s);
    double Sr1b = A.Srb1[i] + Mb * P.rho_w * phi1 * V1 + s_i * Srsb;
    double sbar = Sr1 * Srsb;
    double dJ, dphi, ds;
    swrc_grad(P, J1, phi1, s_i, &dJ, &dphi, &ds);
    const double J1b = A.Jb1[i] + Sr1b * dJ;
    phi1b += Sr1b * dphi;
    sbar += Sr1b * ds;
    const double Jdb = J1b * J0 + V1b * V0 + phi1b * (1.0 - phi0) / (Jd * Jd);
    A.Jb[i] = J1b * Jd;
    A.phib[i] = phi1b / Jd;
    A.sb[i] = sbar;
    Vb_own += V1b * Jd;
    // Jd = 1/det(B), B = I - dt L_i, L_i = N_i K_i^{-1}
    double Ks_i[6] = {0, 0, 0, 0, 0, 0}, Nb_i[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (shape_regular(P.plane != 0, pt, nf) && dt != 0.0) {
      double Ki[6], KiF[9], Li[9], B[9], Bi[9];
      shape_inverse_of(P.plane != 0, pt, Ki);
      sym_full(Ki, KiF);
      mat3_mul(pt + 6, KiF, Li);
      for (int k = 0; k < 9; ++k) B[k] = (k % 4 == 0 ? 1.0 : 0.0) - dt * Li[k];
      const double dB = B[0] * (B[4] * B[8] - B[5] * B[7]) - B[1] * (B[3] * B[8] - B[5] * B[6]) +
                        B[2] * (B[3] * B[7] - B[4] * B[6]);
      Bi[0] = (B[4] * B[8] - B[5] * B[7]) / dB; Bi[1] = (B[2] * B[7] - B[1] * B[8]) / dB;
      Bi[2] = (B[1] * B[5] - B[2] * B[4]) / dB; Bi[3] = (B[5] * B[6] - B[3] * B[8]) / dB;
      Bi[4] = (B[0] * B[8] - B[2] * B[6]) / dB; Bi[5] = (B[2] * B[3] - B[0] * B[5]) / dB;
      Bi[6] = (B[3] * B[7] - B[4] * B[6]) / dB; Bi[7] = (B[1] * B[6] - B[0] * B[7]) / dB;
      Bi[8] = (B[0] * B[4] - B[1] * B[3]) / dB;
      // dJd/dB = -Jd B^{-T};  Lbar = -dt Bbar = dt Jdb Jd B^{-T}
      double Lb[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Lb[3 * r + c] = dt * Jdb * Jd * Bi[3 * c + r];
      mat3_mul(Lb, KiF, Nb_i);
      const double* Ni = pt + 6;
      double NT[9] = {Ni[0], Ni[3], Ni[6], Ni[1], Ni[4], Ni[7], Ni[2], Ni[5], Ni[8]};
      double KibF[9], u9[9], KbF[9], Kbu[6];
      mat3_mul(NT, Lb, KibF);
      mat3_mul(KiF, KibF, u9);
      mat3_mul(u9, KiF, KbF);
      for (int k = 0; k < 9; ++k) KbF[k] = -KbF[k];
      unique_grad(KbF, Kbu);
      sym_full_grad<double>(Kbu, Ks_i);
    }
    for (int k = 0; k < 6; ++k) pt[16 + k] = Ks_i[k];
    for (int k = 0; k < 9; ++k) pt[22 + k] = Nb_i[k];
    pt[31] = Vhb;
    A.own_V[i] = Vb_own;
  }
  __syncthreads();

  // ---- reverse of the sums (R3): G_k = Ks_i + sum_j B_kj Ks_j, H_k = Nb_i + sum_j B_kj Nb_j.
  // The 15 columns [Ks_j | Nb_j] run on the matrix cores; rows k land in
  // sM (columns 0-9), sTb (columns 10-13) and the last slot of sY (column
  // 14), all free by now.
  auto tiles2 = [&](int t0, auto nbc) {
    constexpr int NB = decltype(nbc)::value;
    V4 acc[NB];
    unsigned piece[NB];
    int krow[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[b] = V4{0, 0, 0, 0};
      piece[b] = 0u;
      krow[b] = (t0 + kBondWaves * b) * 16 + r16;
    }
    for (int js = 0; js < nks; ++js) {
      const int j = 4 * js + q4;
      const bool ok = j < nf && r16 < 15;
      const double kv = sKN[16 * (size_t)(ok ? j : 0) + (r16 < 15 ? r16 : 0)];
      const Acc bval = ok ? (Acc)kv : (Acc)0;
      const int s = js & 15;
      if (s == 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const bool rv = krow[b] < nf;
          const unsigned pw = sq[((size_t)(rv ? krow[b] : 0) * nw + (js >> 4)) * 4 + q4];
          piece[b] = rv ? pw : 0u;
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = MM::run((piece[b] >> s) & 1u ? (Acc)1 : (Acc)0, bval, acc[b]);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int t = t0 + kBondWaves * b;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kr = t * 16 + MM::row(q4, r);
        if (kr < nf && r16 < 15) {
          if (r16 < 10) sM[kr].v[r16] = acc[b][r];
          else if (r16 < 14) sTb[kr].v[r16 - 10] = acc[b][r];
          else sY[kr].v[3] = acc[b][r];
        }
      }
    }
  };
  for (int t0 = wid; t0 < ntile; t0 += kBondWaves * kTileBatch) {
    const int nb = (ntile - t0 + kBondWaves - 1) / kBondWaves;
    tile_slots(nb, t0, tiles2);
  }
  __syncthreads();
  double ox[3] = {0, 0, 0}, oy[3] = {0, 0, 0};
  const double Vhb = pt[31];
  for (int m = tid; m < nf; m += kBondThreads) {
    double G[6], H[9];
    const MRec<double> g10 = sM[m];
    const Quad<double> g4 = sTb[m];
    for (int k = 0; k < 6; ++k) G[k] = pt[16 + k] + g10.v[k];
    for (int k = 0; k < 4; ++k) H[k] = pt[22 + k] + g10.v[6 + k];
    for (int k = 0; k < 4; ++k) H[4 + k] = pt[26 + k] + g4.v[k];
    const Quad<double> zq = sZ[m];
    const Quad<double> yq = sY[m];
    H[8] = pt[30] + yq.v[3];
    const double z[3] = {zq.v[0], zq.v[1], zq.v[2]}, y[3] = {yq.v[0], yq.v[1], yq.v[2]};
    const double Vk = zq.v[3];
    double Gz[3], Hz[3], HTy[3];
    symv(G, z, Gz);
    for (int r = 0; r < 3; ++r) Hz[r] = H[3 * r] * z[0] + H[3 * r + 1] * z[1] + H[3 * r + 2] * z[2];
    for (int c = 0; c < 3; ++c) HTy[c] = H[c] * y[0] + H[3 + c] * y[1] + H[6 + c] * y[2];
    const int64_t slot = b0 + m;
    double zbar[3], ybar[3];
    for (int c = 0; c < 3; ++c) {
      zbar[c] = A.slot_x[8 * slot + c] + Vk * (Gz[c] + HTy[c]);
      ybar[c] = Vk * Hz[c];
    }
    const double Vbar = A.slot_V[8 * slot] + 0.5 * (z[0] * Gz[0] + z[1] * Gz[1] + z[2] * Gz[2]) +
                        (y[0] * Hz[0] + y[1] * Hz[1] + y[2] * Hz[2]) + Vhb;
    for (int c = 0; c < 3; ++c) {
      A.slot_x[8 * slot + c] = zbar[c];
      A.slot_vh[8 * slot + c] = ybar[c];
      ox[c] -= zbar[c];
      oy[c] -= ybar[c];
    }
    A.slot_V[8 * slot] = Vbar;
  }
  for (int c = 0; c < 3; ++c) {
    ox[c] = wave_sum(ox[c]);
    oy[c] = wave_sum(oy[c]);
  }
  __syncthreads();
  if (lane == 0)
    for (int c = 0; c < 3; ++c) { red[wid][c] = ox[c]; red[wid][3 + c] = oy[c]; }
  __syncthreads();
  if (tid == 0) {
    for (int c = 0; c < 3; ++c) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < kBondWaves; ++w) { a += red[w][c]; b += red[w][3 + c]; }
      A.own_x[c * n + i] = a;
      A.own_vh[c * n + i] = b;
    }
  }
}

// Per point: collect the contributions other points made to this one
// (stored at slot (i,k), found through rev[]), finish the reverse of the
// predictor, and write the adjoint of state n.
__global__ __launch_bounds__(256) void k_adj_point2(int64_t n, const int64_t* __restrict__ row,
                                                    const int32_t* __restrict__ rev, const uint8_t* __restrict__ fixed,
                                                    const double* __restrict__ own_x, const double* __restrict__ own_vh,
                                                    const double* __restrict__ own_V, const double* __restrict__ slot_x,
                                                    const double* __restrict__ slot_vh,
                                                    const double* __restrict__ slot_V, int64_t cap,
                                                    const double* __restrict__ sigb, const double* __restrict__ pcb,
                                                    const double* __restrict__ Jb, const double* __restrict__ phib,
                                                    const double* __restrict__ sb, ulppm_state In, ulppm_state Out,
                                                    double dt, ContactDev C, bool plane,
                                                    const double* __restrict__ fbar,
                                                    const double* __restrict__ xp, const double* __restrict__ vhp,
                                                    const double* __restrict__ voln) {
  const int lane = threadIdx.x & (kWave - 1);
  const XcdWalk W = xcd_walk(n, 4);
  for (int64_t k = W.first; k < W.end; k += W.stride) {
    double ax[3] = {0, 0, 0}, av[3] = {0, 0, 0}, aV = 0.0;
    for (int64_t s = row[k] + lane; s < row[k + 1]; s += kWave) {
      const double* rec = slot_x + 8 * (int64_t)rev[s];   // the record of slot (k,j) for (j,k)
      for (int c = 0; c < 3; ++c) {
        ax[c] += rec[c];
        av[c] += rec[3 + c];
      }
      aV += rec[6];
    }
    for (int c = 0; c < 3; ++c) {
      ax[c] = wave_sum(ax[c]);
      av[c] = wave_sum(av[c]);
    }
    aV = wave_sum(aV);
    double cx[3] = {0.0, 0.0, 0.0}, cV = 0.0;
    if (C.on) {                                             // contact forces on k (Eqs. 91-93)
      const double fb[3] = {fbar[k], fbar[n + k], fbar[2 * n + k]};
      contact_adjoint(C, plane, xp[k], xp[n + k], xp[2 * n + k], vhp[k], vhp[n + k], vhp[2 * n + k], voln[k], fb,
                      lane, cx, &cV);
      for (int c = 0; c < 3; ++c) cx[c] = wave_sum(cx[c]);
      cV = wave_sum(cV);
    }
    if (lane == 0) {
      const bool fx = fixed[k] != 0, drv = fixed[k] == 2;
      for (int c = 0; c < 3; ++c) {
        const double xb = own_x[c * n + k] + ax[c] + cx[c];
        const double ub = In.u[c][k] + xb;                   // u^{n+1} = u^n + dt v_half, x = x0 + u^{n+1}
        const double vhb = In.v[c][k] + own_vh[c * n + k] + av[c] + dt * ub;
        Out.x0[c][k] = In.x0[c][k] + xb;
        Out.u[c][k] = ub;
        Out.uc[c][k] = -ub;
        // fixed: v_half = 0; driven: v_half = v^n, a = 0; free: v_half = v^n + (dt/2) a^n
        Out.v[c][k] = drv ? vhb : fx ? 0.0 : vhb;
        Out.a[c][k] = fx ? 0.0 : 0.5 * dt * vhb;
      }
      Out.vol[k] = own_V[k] + aV + cV;
      Out.phi[k] = phib[k];
      Out.J[k] = Jb[k];
      Out.Sr[k] = 0.0;
      Out.mass[k] = 0.0;
      Out.s[k] = In.s[k] + sb[k];
      for (int c = 0; c < 6; ++c) Out.sig[c][k] = sigb[c * n + k];
      Out.pc[k] = pcb[k];
    }
  }
}

// Sum of the per-block parameter partials (4 per block) in a fixed order:
// 1024 threads, each folding every 1024th block four at a time, then a tree.
constexpr int kThetaThreads = 1024;
__global__ __launch_bounds__(kThetaThreads) void k_adj_theta(const double* __restrict__ part, int64_t nb,
                                                            double* __restrict__ th) {
  __shared__ double s[4][kThetaThreads];
  double a[4] = {0, 0, 0, 0};
#pragma unroll 4
  for (int64_t b = threadIdx.x; b < nb; b += kThetaThreads)
    for (int k = 0; k < 4; ++k) a[k] += part[4 * b + k];
  for (int k = 0; k < 4; ++k) s[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int o = kThetaThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 0; k < 4; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) th[k] += s[k][0];
}

// Reverse of the point set-up (k_init_points) at the state it produced, S.
// B is the adjoint of that state.  The set-up's nodal force is a function of
// the total stress alone (at dt_inc = 0 the bond stress is the point's
// effective stress, and Eq. 32 adds S_r s 1 back), so the initial
// acceleration a = f/M + g depends on suction only through the mass.  The
// suction adjoint runs through the mass (Eq. 48), the effective stress
// (Eq. 2) and the pre-consolidation (Eqs. 40, 45) into S_r (Eq. 15) and s;
// the pre-consolidation adds the M adjoint.  Four partials per block (M, 0, 0, 0).
__global__ void k_adj_init(ulppm_state S, ulppm_state B, DevParams P, double ocr, double* __restrict__ sbar,
                           double* __restrict__ part) {
  double Mb = 0.0;
  const double g[3] = {P.g0, P.g1, P.g2};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * blockDim.x) {
    const double s = S.s[i], phi = S.phi[i], Sr = S.Sr[i], m = S.mass[i];
    double mb = B.mass[i];
    if (S.fixed[i] == 0)
      for (int c = 0; c < 3; ++c) mb -= B.a[c][i] * (S.a[c][i] - g[c]) / m;
    double Srb = B.Sr[i] + mb * P.rho_w * phi * S.vol[i];
    double sg[6];
    for (int k = 0; k < 6; ++k) sg[k] = S.sig[k][i];
    const double p = (sg[0] + sg[1] + sg[2]) / 3.0;
    const double d[3] = {sg[0] - p, sg[1] - p, sg[2] - p};
    const double q2 = 1.5 * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + 2.0 * (sg[3] * sg[3] + sg[4] * sg[4] + sg[5] * sg[5]));
    const double M2p = P.M * P.M * p;
    const double pcb = ocr * (p + q2 / M2p);
    const double pcbb = B.pc[i] * S.pc[i] / (P.b2 * pcb);     // d pc / d pcb of Eq. 45 inverted
    Mb += pcbb * ocr * (-2.0 * q2 / (M2p * P.M));
    const double dp = ocr * (1.0 - q2 / (M2p * p)), dq = ocr / M2p;
    double tr = 0.0;
    for (int k = 0; k < 3; ++k) tr += B.sig[k][i] + pcbb * (dp / 3.0 + dq * 3.0 * d[k]);
    double dJ, dphi, ds;
    swrc_grad(P, 1.0, phi, s, &dJ, &dphi, &ds);
    Srb -= s * tr;
    sbar[i] = B.s[i] - Sr * tr + Srb * ds;
  }
  __shared__ double r[256];
  r[threadIdx.x] = Mb;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) r[threadIdx.x] += r[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = r[0];
    part[4 * blockIdx.x + 1] = part[4 * blockIdx.x + 2] = part[4 * blockIdx.x + 3] = 0.0;
  }
}

// -------------------------------------------------------- gather kernel --

enum { G_FORCES = 0, G_INIT = 1, G_STEP = 2 };


struct GatherArgs {
  int64_t n, per;
  const int64_t* row;
  const int32_t* col;
  const int32_t* rev;
  const void* T;          // (x, y, z, 0) per bond: double, or float in mixed precision
  const double* vol_n;
  const double* mass;     // M^{n+1}
  const double* vh;       // 3n (G_STEP)
  const uint8_t* fixed;
  double* f[3];           // G_FORCES output
  double* a[3];
  double* v[3];
  double* epart;          // 3 per block (G_STEP)
  unsigned long long* ctr;
  double hdt, g0, g1, g2;
  int mode;
  const double* x;        // 3n current positions (contact)
  ContactDev c;
  int plane;
  const double* fown;     // 3n: sum_j T_ij V_j from the bond kernel, or null (gathered here)
};

// One wave per point: f_i = V_i sum_j (T_ij - T_ji) V_j (Eqs. 49-50, sign of
// Eq. 33), gathering T_ji through rev[] instead of scattering with atomics;
// then a = f/M + g (Eq. 62), v = v_half + (dt/2) a (Eq. 63), energy partials.
// TS: storage and accumulation type of the force gather (float in mixed
// precision); the Newmark update is FP64.  Own: the bond kernel has summed
// each point's own force states (G.fown) and stored V_i T_ik, so only the
// reverse records V_j T_ji are gathered.  LPP: lanes per point, a whole wave,
// or one 16-lane row for families that fit a wave (four points per wave, so
// that the lanes are not left idle by families of a few dozen bonds).
template <class TS, bool Own, int LPP>
__global__ __launch_bounds__(256) void k_gather(GatherArgs G) {
  static_assert(LPP == kWave || LPP == 16, "a point per wave or per 16-lane row");
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int sub = lane & (LPP - 1);                 // lane within the point's group
  const Quad<TS>* T4 = reinterpret_cast<const Quad<TS>*>(G.T);
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  // the sum over the point's group of lanes, left in every lane of the group
  auto group_sum = [](auto v) {
    if constexpr (LPP == kWave) {
      return wave_sum(v);
    } else if constexpr (sizeof(v) == 8) {
      v += dpp_d<kDppXor1, 0xF>(v);
      v += dpp_d<kDppXor2, 0xF>(v);
      v += dpp_d<kDppHalfMirror, 0xF>(v);
      return v + dpp_d<kDppMirror, 0xF>(v);
    } else {
      v += dpp_f<kDppXor1, 0xF>(v);
      v += dpp_f<kDppXor2, 0xF>(v);
      v += dpp_f<kDppHalfMirror, 0xF>(v);
      return v + dpp_f<kDppMirror, 0xF>(v);
    }
  };
  const XcdWalk W = xcd_walk_groups(G.n, 256 / LPP, threadIdx.x / LPP);
  for (int64_t i = W.first; i < W.end; i += W.stride) {
    const int64_t b0 = G.row[i], b1 = G.row[i + 1];
    TS f0 = 0, f1 = 0, f2 = 0;
    if constexpr (Own) {
      // loaded before the bond loop so that the latency overlaps it
      f0 = (TS)G.fown[i];
      f1 = (TS)G.fown[G.n + i];
      f2 = (TS)G.fown[2 * G.n + i];
      if (sub != 0) f0 = f1 = f2 = (TS)0;           // added once by the group sum
      for (int64_t s = b0 + sub; s < b1; s += LPP) {
        const Quad<TS> tr = T4[G.rev[s]];             // V_j T_ji, scaled by point j
        f0 -= tr.v[0];
        f1 -= tr.v[1];
        f2 -= tr.v[2];
      }
    } else {
      for (int64_t s = b0 + sub; s < b1; s += LPP) {
        const int32_t j = G.col[s], r = G.rev[s];
        const TS wv = (TS)G.vol_n[j];
        const Quad<TS> ts = T4[s], tr = T4[r];
        f0 += (ts.v[0] - tr.v[0]) * wv;
        f1 += (ts.v[1] - tr.v[1]) * wv;
        f2 += (ts.v[2] - tr.v[2]) * wv;
      }
    }
    f0 = group_sum(f0);
    f1 = group_sum(f1);
    f2 = group_sum(f2);
    double fc[3] = {0.0, 0.0, 0.0};
    if constexpr (LPP == kWave) {                   // the host runs contact with a wave per point
      if (G.c.on) {
        contact_density(G.c, G.plane != 0, G.x[i], G.x[G.n + i], G.x[2 * G.n + i], G.vh[i], G.vh[G.n + i],
                        G.vh[2 * G.n + i], lane, fc);
        fc[0] = wave_sum(fc[0]);
        fc[1] = wave_sum(fc[1]);
        fc[2] = wave_sum(fc[2]);
      }
    }
    if (sub == 0) {
      const double Vi = G.vol_n[i];
      const double f[3] = {(double)f0 * Vi + Vi * fc[0], (double)f1 * Vi + Vi * fc[1],
                           (double)f2 * Vi + Vi * fc[2]};
      if (G.mode == G_FORCES) {
        for (int c = 0; c < 3; ++c) G.f[c][i] = f[c];
      } else {
        const bool fx = G.fixed[i] != 0;
        const double M = G.mass[i];
        const double g[3] = {G.g0, G.g1, G.g2};
        bool bad = false;
        for (int c = 0; c < 3; ++c) {
          const double a = fx ? 0.0 : f[c] / M + g[c];
          G.a[c][i] = a;
          if (G.mode == G_STEP) {
            const double vhc = G.vh[c * G.n + i];
            const double v = vhc + G.hdt * a;
            G.v[c][i] = v;
            if (!fx) {
              e0 -= G.hdt * vhc * f[c];
              e1 += G.hdt * vhc * M * g[c];
            }
            e2 += 0.5 * M * v * v;
            bad = bad || !isfinite(v);
          }
          bad = bad || !isfinite(a);
        }
        if (bad) ctr_add(G.ctr, C_NONFINITE, 1ull);
      }
    }
  }
  if (G.mode == G_STEP) {
    if constexpr (LPP != kWave) {                   // the groups' partials
      e0 = wave_sum(e0);
      e1 = wave_sum(e1);
      e2 = wave_sum(e2);
    }
    __shared__ double r[3][4];
    if (lane == 0) { r[0][wid] = e0; r[1][wid] = e1; r[2][wid] = e2; }
    __syncthreads();
    if (threadIdx.x == 0) {
      G.epart[3 * blockIdx.x + 0] = r[0][0] + r[0][1] + r[0][2] + r[0][3];
      G.epart[3 * blockIdx.x + 1] = r[1][0] + r[1][1] + r[1][2] + r[1][3];
      G.epart[3 * blockIdx.x + 2] = r[2][0] + r[2][1] + r[2][2] + r[2][3];
    }
  }
}

// Deterministic energy totals: one block sums the per-block partials of the
// predictor (2 per block) and of the gather (3 per block) in a fixed order.
__global__ void k_energy(const double* __restrict__ pp, int npb, const double* __restrict__ gp, int ngb,
                         double* __restrict__ E, const int64_t* __restrict__ row, int64_t n,
                         unsigned long long* __restrict__ ctr) {
  __shared__ double s[3][256];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < npb; k += 256) { a += pp[2 * k]; b += pp[2 * k + 1]; }
  for (int k = threadIdx.x; k < ngb; k += 256) { a += gp[3 * k]; b += gp[3 * k + 1]; c += gp[3 * k + 2]; }
  s[0][threadIdx.x] = a; s[1][threadIdx.x] = b; s[2][threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 3; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    E[0] += s[0][0];
    E[1] += s[1][0];
    E[2] = s[2][0];
    ctr[C_BONDSUM * kStripes] += (unsigned long long)row[n];   // single thread, stream-ordered
  }
}

// -------------------------------------------------------- init / dt_crit --

// Point set-up of the initial conditions (Algorithm 2): J = 1, u = 0,
// Sr from Eq. 15 at J = 1, effective stress = total - Sr s 1 (Eq. 2,
// p_w = -s), pre-consolidation = ocr times the isotropic intercept of the
// yield surface through that stress (Eq. 40), inverted through Eq. 45;
// mass from Eq. 48.
__global__ void k_init_points(ulppm_state S, DevParams P, double ocr) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S.n; i += (int64_t)gridDim.x * blockDim.x) {
    S.J[i] = 1.0;
    for (int c = 0; c < 3; ++c) { S.u[c][i] = 0.0; S.uc[c][i] = 0.0; }
    const double s = S.s[i], phi = S.phi[i];
    const double Sr = swrc(P, 1.0, phi, s);
    S.Sr[i] = Sr;
    double sg[6];
    for (int k = 0; k < 6; ++k) sg[k] = S.sig[k][i] - (k < 3 ? Sr * s : 0.0);
    for (int k = 0; k < 6; ++k) S.sig[k][i] = sg[k];
    const double p = (sg[0] + sg[1] + sg[2]) / 3.0;
    const double d0 = sg[0] - p, d1 = sg[1] - p, d2 = sg[2] - p;
    const double q2 = 1.5 * (d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * (sg[3] * sg[3] + sg[4] * sg[4] + sg[5] * sg[5]));
    const double pcb = ocr * (p + q2 / (P.M * P.M * p));
    S.pc[i] = -pow(-pcb * exp(-P.b1), 1.0 / P.b2);
    S.mass[i] = (P.rho_s * (1.0 - phi) + P.rho_w * Sr * phi) * S.vol[i];
  }
}

// Eq. 65 per point (C/|zeta| with C = 18 K / (pi delta^4)); block minima.
__global__ void k_dtcrit(int64_t n, const int64_t* __restrict__ row, const int32_t* __restrict__ col,
                         const double* __restrict__ x, const double* __restrict__ vol,
                         const double* __restrict__ phi, double C, double rho_s, double* __restrict__ part) {
  double best = INFINITY;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double sum = 0.0;
    for (int64_t s = row[i]; s < row[i + 1]; ++s) {
      const int32_t j = col[s];
      const double z = sqrt(exact_r2(x[i], x[n + i], x[2 * n + i], x[j], x[n + j], x[2 * n + j]));
      sum += vol[j] * C / z;
    }
    if (sum > 0.0) best = fmin(best, sqrt(2.0 * (1.0 - phi[i]) * rho_s / sum));
  }
  __shared__ double s[256];
  s[threadIdx.x] = best;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = fmin(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Folds the counter stripes: sums, except the maxima.
// One wave per counter: each lane folds every 64th stripe, then the wave.
__global__ __launch_bounds__(C_NCOUNT * kWave) void k_reduce_counters(const unsigned long long* __restrict__ ctr,
                                                                     unsigned long long* __restrict__ out) {
  const int k = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const bool is_max = k == C_MAXNEWTON || k == C_MAXFAM;
  unsigned long long a = 0;
  for (int t = lane; t < kStripes; t += kWave) {
    const unsigned long long v = ctr[k * kStripes + t];
    a = is_max ? (a > v ? a : v) : a + v;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(a, off);
    a = is_max ? (a > o ? a : o) : a + o;
  }
  if (lane == 0) out[k] = a;
}

__global__ void k_export_rows(int64_t n, const int64_t* __restrict__ row, int64_t* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e <= n; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = row[e];
}

__global__ void k_copy_i32(const int32_t* __restrict__ a, int32_t* __restrict__ b, int64_t m) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
    b[e] = a[e];
}

// One component of the per-bond force-state records, widened to double.
template <class TS>
__global__ void k_unpack_T(const Quad<TS>* __restrict__ T, int c, double* __restrict__ b, int64_t m) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
    b[e] = (double)T[e].v[c];
}
// The same from records that hold V_i T_ik (the FP64 path with own sums):
// one thread per point i divides its row by V_i.
__global__ void k_unpack_T_scaled(const Quad<double>* __restrict__ T, int c, const int64_t* __restrict__ row,
                                  const double* __restrict__ vol, int64_t n, double* __restrict__ b) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double Vi = vol[i];
    for (int64_t e = row[i]; e < row[i + 1]; ++e) b[e] = T[e].v[c] / Vi;
  }
}

__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, int64_t m) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
    b[e] = a[e];
}

}  // namespace

// ==================================================================== host ==

struct ulppm_ctx {
  hipStream_t stream = nullptr;
  int64_t cap_n = 0;
  int max_f = 0;
  int seen_max_f = 0;       // largest family any call on this context has reported
  int64_t max_cells = 0;
  int64_t bond_cap = 0;
  // per point
  double* x = nullptr;      // 3n
  double* vh = nullptr;     // 3n
  double* vol_n = nullptr;  // n
  double* pscr = nullptr;   // 12n point scratch for non-mutating passes
  double* pk = nullptr;     // 2n per-point values of the bond pass
  double* xv = nullptr;     // 8n packed x, V^n, v_half per point (bond-pass gathers)
  double* fown = nullptr;   // 3n own-row force sums of the bond kernel (FP64)
  int32_t* cellid = nullptr;
  int32_t* cnt = nullptr;
  int64_t* row = nullptr;   // n+1
  // candidate lists (radius delta + skin), rebuilt only when needed
  int max_c = 0;
  int32_t* cand = nullptr;    // n*max_c, rows ascending
  int32_t* ccnt = nullptr;    // n
  int32_t* crev = nullptr;    // n*max_c, position of i in the candidate row of j
  unsigned long long* fbits = nullptr;  // n*max_c/64: membership bit of each candidate slot
  double* xref = nullptr;     // 3n positions at the last candidate build
  int32_t* gate = nullptr;    // 1: rebuild candidates in this step
  int64_t built_n = -1;       // point count and horizon of the last candidate build
  double built_delta = 0.0;
  // cells
  int32_t* ccount = nullptr;
  int32_t* ccursor = nullptr;
  int64_t* cstart = nullptr;  // max_cells+1
  int32_t* cpts = nullptr;    // n
  // bonds
  int32_t* col = nullptr;
  int32_t* rev = nullptr;
  double* T = nullptr;        // 4*bond_cap: (x, y, z, 0) per bond, double or float
  // reductions
  double* part = nullptr;     // partials
  int64_t part_cap = 0;
  int64_t* scan_bsum = nullptr;
  int64_t scan_cap = 0;
  Grid* grid = nullptr;
  unsigned long long* ctr = nullptr;      // C_NCOUNT x kStripes
  unsigned long long* ctr_sum = nullptr;  // C_NCOUNT, folded
  double* E = nullptr;        // 3
  ContactDev contact = {};    // substrate (ulppm_set_contact); off by default
  // history on the bonds (ulppm_history_reserve): hist[last] holds the states
  // of the last step in the order of hist_row/hist_col, 8 doubles per bond
  double* hist[2] = {nullptr, nullptr};
  int64_t* hist_row = nullptr;
  int32_t* hist_col = nullptr;
  int64_t* hist_map = nullptr; // per bond slot: slot of the same bond in the previous families, or -1
  int hist_last = 0;
  int64_t hist_n = 0;         // points of the held history; 0: none
  // adjoint scratch (ulppm_adjoint_reserve)
  double* adj = nullptr;      // 24n forward copy + 21n point adjoints + 4(n+8) partials
  double* adj_slot = nullptr; // 16 x bond_cap: adjoint slot records (8), bond tail forward solutions (8)
  double* adj_hist = nullptr; // 16 x bond_cap: carried start states and their adjoints (history on the bonds)
  // phase timing events, [step][phase][start/stop]
  hipEvent_t ev[kTimedSteps][kPhases][2] = {};
  bool have_events = false;
  // host mirrors
  unsigned long long h_ctr[C_NCOUNT];
  std::string err;
};

namespace {

int fail(ulppm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(call)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail(ctx, ULPPM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

DevParams dev_params(const ulppm_params* p) {
  DevParams d;
  d.delta = p->delta;
  d.d2 = p->delta * p->delta;
  d.K = p->K; d.mu = p->mu; d.M = p->M; d.lam = p->lam; d.kap = p->kap; d.eta = p->eta;
  d.b1 = p->b1; d.b2 = p->b2; d.rho_s = p->rho_s; d.rho_w = p->rho_w;
  d.a1 = p->a1; d.a2 = p->a2; d.n_vg = p->n_vg;
  d.g0 = p->g[0]; d.g1 = p->g[1]; d.g2 = p->g[2];
  d.dt = p->dt;
  d.newton_tol = p->newton_tol;
  d.newton_maxit = p->newton_maxit;
  d.force_mode = p->force_mode;
  d.iM2 = 1.0 / (p->M * p->M);
  d.plane = p->plane;
  return d;
}

int check_state(ulppm_ctx* ctx, const ulppm_state* S) {
  if (!S) return fail(ctx, ULPPM_E_ARG, "state is NULL");
  if (S->n <= 0 || S->n > ctx->cap_n) return fail(ctx, ULPPM_E_ARG, "state n out of range for this context");
  for (int c = 0; c < 3; ++c)
    if (!S->x0[c] || !S->u[c] || !S->uc[c] || !S->v[c] || !S->a[c]) return fail(ctx, ULPPM_E_ARG, "NULL vector field");
  for (int k = 0; k < 6; ++k)
    if (!S->sig[k]) return fail(ctx, ULPPM_E_ARG, "NULL stress component");
  if (!S->vol || !S->phi || !S->J || !S->Sr || !S->mass || !S->s || !S->pc || !S->fixed)
    return fail(ctx, ULPPM_E_ARG, "NULL scalar field");
  return ULPPM_OK;
}

int check_params(ulppm_ctx* ctx, const ulppm_params* p) {
  if (!p) return fail(ctx, ULPPM_E_ARG, "params is NULL");
  if (!(p->delta > 0.0) || !std::isfinite(p->delta)) return fail(ctx, ULPPM_E_ARG, "delta must be > 0");
  if (!(p->K > 0.0) || !(p->mu > 0.0) || !(p->M > 0.0) || !(p->eta > 0.0) || !(p->lam > p->kap))
    return fail(ctx, ULPPM_E_ARG, "material constants out of range");
  if (p->newton_maxit < 1 || p->newton_maxit > 1000) return fail(ctx, ULPPM_E_ARG, "newton_maxit out of range");
  if (p->precision != ULPPM_FP64 && p->precision != ULPPM_MIXED) return fail(ctx, ULPPM_E_ARG, "bad precision");
  if (p->force_mode != ULPPM_FORCE_CONJUGATE && p->force_mode != ULPPM_FORCE_EQ51 &&
      p->force_mode != ULPPM_FORCE_STANDARD)
    return fail(ctx, ULPPM_E_ARG, "bad force_mode");
  if (p->plane != 0 && p->plane != 1) return fail(ctx, ULPPM_E_ARG, "plane must be 0 or 1");
  if (p->history != ULPPM_HISTORY_POINT && p->history != ULPPM_HISTORY_BOND)
    return fail(ctx, ULPPM_E_ARG, "bad history");
  if (p->history == ULPPM_HISTORY_BOND && p->force_mode == ULPPM_FORCE_STANDARD)
    return fail(ctx, ULPPM_E_ARG, "the standard model has no bond stresses to carry");
  return ULPPM_OK;
}

// Grid for the per-point kernels that walk points with xcd_walk: 4 waves per
// block, at most 2 points per wave per pass, a multiple of 8 blocks, capped.
inline unsigned walk_grid(int64_t n) {
  int64_t b = (n + 7) / 8;
  b = std::min<int64_t>(std::max<int64_t>(b, 1), 512);
  return (unsigned)(8 * b);
}

inline int blocks_for(int64_t n, int t, int cap = 65536) {
  int64_t b = (n + t - 1) / t;
  if (b < 1) b = 1;
  return (int)(b > cap ? cap : b);
}

int zero_counters(ulppm_ctx* ctx) {
  k_fill<unsigned long long><<<16, 256, 0, ctx->stream>>>(ctx->ctr, C_NCOUNT * kStripes, 0ull);
  HIPCHK(hipGetLastError());
  return ULPPM_OK;
}

int scan_counts(ulppm_ctx* ctx, const int32_t* cnt, int64_t m, int64_t* out, const int32_t* gate = nullptr) {
  const int64_t nb = (m + kScanChunk - 1) / kScanChunk;
  if (nb > ctx->scan_cap) return fail(ctx, ULPPM_E_ARG, "scan too large");
  if (nb == 0) {
    k_fill<int64_t><<<1, 64, 0, ctx->stream>>>(out, 1, 0, gate);
    HIPCHK(hipGetLastError());
    return ULPPM_OK;
  }
  k_scan_blocks<<<(unsigned)nb, 256, 0, ctx->stream>>>(cnt, m, out, ctx->scan_bsum, gate);
  k_scan_top<<<1, 1024, 0, ctx->stream>>>(ctx->scan_bsum, nb, out, m, gate);
  k_scan_add<<<(unsigned)nb, 256, 0, ctx->stream>>>(out, m, ctx->scan_bsum, gate);
  HIPCHK(hipGetLastError());
  return ULPPM_OK;
}

// Families at the positions in ctx->x (Eq. 1).  Candidate lists within
// delta + skin are rebuilt on the device when the gate is set (force, or a
// point moved more than skin/2 since the last build); every step then
// filters the candidates with the exact predicate, so the families are
// exactly those of the current positions.  Then CSR offsets and rev[].
// Candidate lists are rebuilt when forced, when the point count or horizon
// changed since the last build, or when a point has left half the skin.
int build_families(ulppm_ctx* ctx, int64_t n, double delta, bool force) {
  const double skin = kSkin * delta;
  const double rc = delta + skin;
  const int32_t* gate = ctx->gate;
  force = force || ctx->built_n != n || ctx->built_delta != delta;
  ctx->built_n = n;
  ctx->built_delta = delta;
  if (force) {
    k_fill<int32_t><<<1, 64, 0, ctx->stream>>>(ctx->gate, 1, 1);
  } else {
    const double half = 0.5 * skin * (1.0 - 1e-6);
    k_check_skin<<<blocks_for(n, 256, 2048), 256, 0, ctx->stream>>>(ctx->x, ctx->xref, n, half * half, ctx->gate);
  }
  const int nbb = blocks_for(n, 256, 1024);
  k_bbox<<<nbb, 256, 0, ctx->stream>>>(ctx->x, n, ctx->part + kPartRed, gate);
  k_grid<<<1, 256, 0, ctx->stream>>>(ctx->part + kPartRed, nbb, rc, ctx->max_cells, ctx->grid, ctx->ctr, gate);
  k_fill<int32_t><<<blocks_for(ctx->max_cells, 256, 4096), 256, 0, ctx->stream>>>(ctx->ccount, ctx->max_cells, 0, gate);
  k_fill<int32_t><<<blocks_for(ctx->max_cells, 256, 4096), 256, 0, ctx->stream>>>(ctx->ccursor, ctx->max_cells, 0, gate);
  k_cell_count<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(ctx->x, n, ctx->grid, ctx->cellid, ctx->ccount, gate);
  HIPCHK(hipGetLastError());
  int rc2 = scan_counts(ctx, ctx->ccount, ctx->max_cells, ctx->cstart, gate);
  if (rc2) return rc2;
  k_cell_fill<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, ctx->cellid, ctx->cstart, ctx->ccursor, ctx->cpts, gate);
  const int64_t per = (n + 7) / 8;
  // capped grids: most steps the gate is clear and every block returns at once,
  // so the launch cost is that of dispatching the blocks
  const unsigned fgrid = (unsigned)std::min<int64_t>(8 * per, 4096);
  k_family<<<fgrid, kWave, ctx->max_c * sizeof(int32_t), ctx->stream>>>(
      ctx->x, n, per, ctx->grid, ctx->cellid, ctx->cstart, ctx->cpts, rc * rc, ctx->max_c, ctx->cand, ctx->ccnt,
      ctx->ctr, gate);
  const unsigned cgrid = (unsigned)((n * ctx->max_c + 255) / 256);
  k_cand_rev<<<std::min<unsigned>(cgrid, 2048u), 256, 0, ctx->stream>>>(n, ctx->max_c, ctx->cand, ctx->ccnt,
                                                                       ctx->crev, ctx->ctr, gate);
  k_save_ref<<<blocks_for(3 * n, 256, 4096), 256, 0, ctx->stream>>>(ctx->x, ctx->xref, 3 * n, ctx->ctr, gate);
  k_fill<int32_t><<<1, 64, 0, ctx->stream>>>(ctx->gate, 1, 0);
  HIPCHK(hipGetLastError());
  // the packed point records carry the positions the filter reads
  k_pack<<<blocks_for(n, 256, 8192), 256, 0, ctx->stream>>>(n, ctx->x, ctx->vh, ctx->vol_n, ctx->xv);
  // candidate lists of a few dozen (families that fit a wave): a 16-lane row
  // per point (P1: 2.94 -> 2.85 ms per step against a wave); lists of about
  // 150 (C1): half a wave per point, two points per wave, in both kernels
  // (family phase 0.279 -> 0.246 ms against a wave, whose last pass over a
  // list leaves most lanes idle; 16 lanes take too many passes)
  const bool rows = ctx->max_f <= kWave;
  if (rows)
    k_filter<16><<<walk_grid(n), 256, 0, ctx->stream>>>(ctx->xv, n, ctx->max_c, ctx->max_f, ctx->cand, ctx->ccnt,
                                                        delta * delta, ctx->fbits, ctx->cnt, ctx->ctr);
  else
    k_filter<32><<<walk_grid(n), 256, 0, ctx->stream>>>(ctx->xv, n, ctx->max_c, ctx->max_f, ctx->cand, ctx->ccnt,
                                                        delta * delta, ctx->fbits, ctx->cnt, ctx->ctr);
  HIPCHK(hipGetLastError());
  rc2 = scan_counts(ctx, ctx->cnt, n, ctx->row);
  if (rc2) return rc2;
  if (rows)
    k_compact<16><<<walk_grid(n), 256, 0, ctx->stream>>>(n, ctx->max_c, ctx->max_f, ctx->cand, ctx->ccnt, ctx->crev,
                                                         ctx->fbits, ctx->row, ctx->col, ctx->rev, ctx->ctr);
  else
    k_compact<32><<<walk_grid(n), 256, 0, ctx->stream>>>(n, ctx->max_c, ctx->max_f, ctx->cand, ctx->ccnt, ctx->crev,
                                                         ctx->fbits, ctx->row, ctx->col, ctx->rev, ctx->ctr);
  HIPCHK(hipGetLastError());
  return ULPPM_OK;
}

// Whether the bond kernel sums each point's own force states for the gather:
// the FP64 conjugate and Eq. 51 paths with families of more than one wave (with small
// families the gather's per-point work is dominated by latency, not by the
// records this saves).
static bool own_sums(const ulppm_ctx* ctx, const ulppm_params* p) {
  return p->precision != ULPPM_MIXED &&
         (p->force_mode == ULPPM_FORCE_CONJUGATE || p->force_mode == ULPPM_FORCE_EQ51) && ctx->max_f > kWave;
}

size_t bond_lds(int max_f, bool mixed, int nt) {
  return mixed ? bond_mx_lds_bytes<float>(max_f, nt) : bond_mx_lds_bytes<double>(max_f, nt);
}
// Waves per SIMD the bond kernel's LDS (lds bytes per workgroup of nt
// threads) admits, capped at the instances built: three for FP64 (reached
// from five workgroups of two waves, 2.5 waves per SIMD on average, where the
// third wave still pays), four for mixed precision.
int bond_waves(size_t lds, int nt, bool mixed) {
  const int wg = (int)(kCuLds / (lds + kBondStaticLds));       // workgroups per CU
  const int waves = wg * (nt / kWave);                          // per CU, four SIMDs
  if (mixed) return waves >= 16 ? 4 : 3;
  return waves >= 10 ? 3 : 2;
}

// Launch of the bond kernel: the instance for the precision (Acc), the
// bond-history mode and the pre-consolidation law (LinP), at the workgroup
// width and waves per SIMD that the family capacity admits.  The history
// instances always run two waves.
struct BondLaunch {
  unsigned grid;
  int nt;
  size_t lds;
  hipStream_t stream;
  bool one_wave, more;
};
template <class Acc, bool Hist, bool LinP>
void launch_bond(const BondLaunch& L, const BondArgs& A, const DevParams& P) {
  constexpr int lo = sizeof(Acc) == 8 ? 2 : 3;                   // waves per SIMD without "more"
  if constexpr (!Hist) {
    if (L.one_wave) {
      if (L.more) k_bond_mx<Acc, Hist, LinP, kWave, lo + 1><<<L.grid, L.nt, L.lds, L.stream>>>(A, P);
      else k_bond_mx<Acc, Hist, LinP, kWave, lo><<<L.grid, L.nt, L.lds, L.stream>>>(A, P);
      return;
    }
  }
  if (L.more) k_bond_mx<Acc, Hist, LinP, kBondThreads, lo + 1><<<L.grid, L.nt, L.lds, L.stream>>>(A, P);
  else k_bond_mx<Acc, Hist, LinP, kBondThreads, lo><<<L.grid, L.nt, L.lds, L.stream>>>(A, P);
}
// The dynamic LDS cap of every instance launch_bond<Acc, Hist, LinP> can pick.
template <class Acc, bool Hist, bool LinP>
void bond_lds_limit(int lds) {
  constexpr int lo = sizeof(Acc) == 8 ? 2 : 3;
  const void* ks[4] = {(const void*)k_bond_mx<Acc, Hist, LinP, kBondThreads, lo>,
                       (const void*)k_bond_mx<Acc, Hist, LinP, kBondThreads, lo + 1>, nullptr, nullptr};
  if constexpr (!Hist) {
    ks[2] = (const void*)k_bond_mx<Acc, Hist, LinP, kWave, lo>;
    ks[3] = (const void*)k_bond_mx<Acc, Hist, LinP, kWave, lo + 1>;
  }
  for (const void* k : ks)
    if (k) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

// Algorithm 1 (bond pass) into outputs; mode: step (state outputs) or not.
// mark(0) / mark(1) bracket the point-kinematics kernels when timing.
int bond_pass(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_params* p, double dt_inc, bool commit,
              const std::function<void(int)>& mark = nullptr, double* hist = nullptr) {
  const int64_t n = S->n;
  BondArgs A;
  A.n = n;
  A.per = (n + 7) / 8;
  A.row = ctx->row;
  A.col = ctx->col;
  A.x = ctx->x;
  A.vh = ctx->vh;
  A.vol_n = ctx->vol_n;
  A.J = S->J;
  A.phi = S->phi;
  A.s = S->s;
  for (int k = 0; k < 6; ++k) A.sig[k] = S->sig[k];
  A.pc = S->pc;
  if (commit) {
    A.J_out = S->J; A.vol_out = S->vol; A.phi_out = S->phi; A.Sr_out = S->Sr; A.mass_out = S->mass;
    for (int k = 0; k < 6; ++k) A.sig_out[k] = S->sig[k];
    A.pc_out = S->pc;
  } else {
    double* q = ctx->pscr;
    A.J_out = q; A.vol_out = q + n; A.phi_out = q + 2 * n; A.Sr_out = q + 3 * n; A.mass_out = q + 4 * n;
    for (int k = 0; k < 6; ++k) A.sig_out[k] = q + (5 + k) * n;
    A.pc_out = q + 11 * n;
  }
  const bool mixed = p->precision == ULPPM_MIXED;
  A.T = ctx->T;
  A.hist = hist;
  A.hist_old = hist ? ctx->hist[ctx->hist_last] : nullptr;
  A.hmap = hist ? ctx->hist_map : nullptr;
  A.fown = own_sums(ctx, p) ? ctx->fown : nullptr;
  A.dt_inc = dt_inc;
  A.max_f = ctx->max_f;
  A.ctr = ctx->ctr;
  A.pk = ctx->pk;
  A.xv = ctx->xv;
  DevParams P = dev_params(p);
  if (mark) mark(0);
  const bool one_wave = ctx->max_f <= kWave;             // every family fits one wave
  const int nt = one_wave && !hist ? kWave : kBondThreads;  // the history instances run two waves
  const size_t lds = bond_lds(ctx->max_f, mixed, nt);
  k_pack<<<blocks_for(n, 256, 8192), 256, 0, ctx->stream>>>(n, ctx->x, ctx->vh, ctx->vol_n, ctx->xv);
  // the standard model's return map lives in its own instance so that the
  // plain kinematics keep their small register footprint
  const bool standard = p->force_mode == ULPPM_FORCE_STANDARD;
  if (mixed && standard)
    k_point_kin_standard<float><<<walk_grid(n), 256, 0, ctx->stream>>>(A, P);
  else if (standard)
    k_point_kin_standard<double><<<walk_grid(n), 256, 0, ctx->stream>>>(A, P);
  else {
    const int64_t per = ((n + kKinPoints - 1) / kKinPoints + 7) / 8;
    k_point_kin_quad<<<(unsigned)(8 * per), 256, 0, ctx->stream>>>(A, P, per);
  }
  if (mark) mark(1);
  if (p->force_mode == ULPPM_FORCE_STANDARD) {
    HIPCHK(hipGetLastError());
    return ULPPM_OK;
  }
  const unsigned grid = (unsigned)(8 * A.per);
  const bool more = bond_waves(lds, nt, mixed) > (mixed ? 3 : 2);
  const bool lin = p->b1 == 0.0 && p->b2 == 1.0;        // Eq. 45 reduces to P = p_c
  const BondLaunch L{grid, nt, lds, ctx->stream, one_wave, more};
  if (mixed && hist) lin ? launch_bond<float, true, true>(L, A, P) : launch_bond<float, true, false>(L, A, P);
  else if (mixed) lin ? launch_bond<float, false, true>(L, A, P) : launch_bond<float, false, false>(L, A, P);
  else if (hist) lin ? launch_bond<double, true, true>(L, A, P) : launch_bond<double, true, false>(L, A, P);
  else lin ? launch_bond<double, false, true>(L, A, P) : launch_bond<double, false, false>(L, A, P);
  HIPCHK(hipGetLastError());
  return ULPPM_OK;
}

int gather_pass(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_params* p, int mode, const double* mass,
                double* const* fout) {
  const int64_t n = S->n;
  GatherArgs G;
  G.n = n;
  G.per = 0;
  G.row = ctx->row;
  G.col = ctx->col;
  G.rev = ctx->rev;
  const bool mixed = p->precision == ULPPM_MIXED;
  G.T = ctx->T;
  G.vol_n = ctx->vol_n;
  G.mass = mass;
  G.vh = ctx->vh;
  G.fixed = S->fixed;
  for (int c = 0; c < 3; ++c) {
    G.f[c] = fout ? fout[c] : nullptr;
    G.a[c] = S->a[c];
    G.v[c] = S->v[c];
  }
  G.epart = ctx->part + kPartGather;
  G.ctr = ctx->ctr;
  G.hdt = 0.5 * p->dt;
  G.g0 = p->g[0]; G.g1 = p->g[1]; G.g2 = p->g[2];
  G.mode = mode;
  G.x = ctx->x;
  G.c = ctx->contact;
  G.plane = p->plane;
  G.fown = own_sums(ctx, p) ? ctx->fown : nullptr;
  const unsigned grid = walk_grid(n);
  if (mode == G_STEP && (int64_t)grid * 3 + kPartGather > ctx->part_cap) return fail(ctx, ULPPM_E_ARG, "partials too small");
  // families that fit a wave: a 16-lane row per point (no contact: its site
  // loop runs over a wave's lanes); the own sums come only with larger ones
  const bool rows = ctx->max_f <= kWave && !G.c.on;
  if (mixed && rows)
    k_gather<float, false, 16><<<grid, 256, 0, ctx->stream>>>(G);
  else if (mixed)
    k_gather<float, false, kWave><<<grid, 256, 0, ctx->stream>>>(G);
  else if (G.fown)
    k_gather<double, true, kWave><<<grid, 256, 0, ctx->stream>>>(G);
  else if (rows)
    k_gather<double, false, 16><<<grid, 256, 0, ctx->stream>>>(G);
  else
    k_gather<double, false, kWave><<<grid, 256, 0, ctx->stream>>>(G);
  HIPCHK(hipGetLastError());
  return ULPPM_OK;
}

int read_counters(ulppm_ctx* ctx) {
  k_reduce_counters<<<1, C_NCOUNT * kWave, 0, ctx->stream>>>(ctx->ctr, ctx->ctr_sum);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(ctx->h_ctr, ctx->ctr_sum, sizeof(ctx->h_ctr), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->seen_max_f = std::max<int>(ctx->seen_max_f, (int)ctx->h_ctr[C_MAXFAM]);
  return ULPPM_OK;
}

int counters_to_status(ulppm_ctx* ctx) {
  if (ctx->h_ctr[C_OVERFLOW])
    return fail(ctx, ULPPM_E_CAPACITY, "a family exceeded max_family=" + std::to_string(ctx->max_f) +
                                           " (largest " + std::to_string(ctx->h_ctr[C_MAXFAM]) + ")");
  if (ctx->h_ctr[C_NONFINITE]) return fail(ctx, ULPPM_E_NONFINITE, "non-finite positions, velocities or accelerations");
  if (ctx->h_ctr[C_ADJLDS])
    return fail(ctx, ULPPM_E_CAPACITY, "adjoint: a family larger than any the forward calls reported");
  if (ctx->h_ctr[C_NOCONV])
    return fail(ctx, ULPPM_E_NOCONV, std::to_string(ctx->h_ctr[C_NOCONV]) + " return-map Newton solves did not converge");
  return ULPPM_OK;
}

void fill_report(ulppm_ctx* ctx, int64_t n, ulppm_report* rep, int64_t steps) {
  if (!rep) return;
  double E[3] = {0, 0, 0};
  int64_t nb = 0;
  (void)hipMemcpyAsync(E, ctx->E, sizeof(E), hipMemcpyDeviceToHost, ctx->stream);
  (void)hipMemcpyAsync(&nb, ctx->row + n, sizeof(nb), hipMemcpyDeviceToHost, ctx->stream);
  (void)hipStreamSynchronize(ctx->stream);
  rep->W_int = E[0];
  rep->W_ext = E[1];
  rep->W_kin = E[2];
  rep->n_bonds = nb;
  rep->n_degenerate = (int64_t)ctx->h_ctr[C_DEGEN];
  rep->n_plastic = (int64_t)ctx->h_ctr[C_PLASTIC];
  rep->max_newton = (int64_t)ctx->h_ctr[C_MAXNEWTON];
  rep->n_noconv = (int64_t)ctx->h_ctr[C_NOCONV];
  rep->n_tests = (int64_t)ctx->h_ctr[C_TESTS];
  rep->n_triples = (int64_t)ctx->h_ctr[C_TRIPLES];
  rep->max_family = (int64_t)ctx->h_ctr[C_MAXFAM];
  rep->steps = steps;
  rep->n_bond_updates = (int64_t)ctx->h_ctr[C_BONDSUM];
  rep->n_rebuilds = (int64_t)ctx->h_ctr[C_REBUILD];
  rep->timed_steps = 0;
  rep->t_predict_ms = rep->t_family_ms = rep->t_bond_ms = rep->t_gather_ms = rep->t_kin_ms = 0.0;
}

// Sum the phase durations of the timed steps of the last ulppm_step call.
void add_timings(ulppm_ctx* ctx, int64_t timed, ulppm_report* rep) {
  if (!rep || timed <= 0) return;
  double t[kPhases] = {0, 0, 0, 0, 0};
  for (int64_t k = 0; k < timed; ++k)
    for (int ph = 0; ph < kPhases; ++ph) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ctx->ev[k][ph][0], ctx->ev[k][ph][1]) == hipSuccess) t[ph] += ms;
    }
  rep->timed_steps = timed;
  rep->t_predict_ms = t[0];
  rep->t_family_ms = t[1];
  rep->t_bond_ms = t[2];
  rep->t_gather_ms = t[3];
  rep->t_kin_ms = t[4];
}

}  // namespace

// =============================================================== C ABI ==

extern "C" {

// Host-only check of the hand-written reverse of the per-bond tail against
// central finite differences (no GPU call).  Random sums, stresses and
// velocity gradients; cases alternate between the elastic and the plastic
// branch.  *max_rel receives the largest relative gradient error, *n_plastic
// the number of plastic cases checked.
int ulppm_selfcheck_tail(const ulppm_params* p, int32_t seed, int32_t n_cases, double* max_rel,
                         int32_t* n_plastic) {
  if (!p || !max_rel || !n_plastic || n_cases <= 0) return ULPPM_E_ARG;
  DevParams P = dev_params(p);
  uint64_t st = 0x9E3779B97F4A7C15ull ^ (uint64_t)seed;
  auto rnd = [&]() {
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    return (double)(st >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  };
  double worst = 0.0;
  int npl = 0;
  for (int cs = 0; cs < n_cases; ++cs) {
    // inputs
    double K[6] = {0, 0, 0, 0, 0, 0};
    for (int m = 0; m < 12; ++m) {
      const double z[3] = {rnd() * 0.03, rnd() * 0.03, rnd() * 0.03};
      K[0] += 1e-6 * z[0] * z[0]; K[1] += 1e-6 * z[1] * z[1]; K[2] += 1e-6 * z[2] * z[2];
      K[3] += 1e-6 * z[1] * z[2]; K[4] += 1e-6 * z[0] * z[2]; K[5] += 1e-6 * z[0] * z[1];
    }
    const bool plastic = (cs % 2) == 1;
    const double gscale = plastic ? 40.0 : 0.5;        // velocity-gradient magnitude [1/s]
    double Ki[6];
    sym_inverse(K, Ki);
    double KiF[9], Lr[9], N[9];
    sym_full(Ki, KiF);
    for (int k = 0; k < 9; ++k) Lr[k] = gscale * rnd();
    // N = L K so that L = N K^{-1} has the chosen size
    double KF[9];
    sym_full(K, KF);
    mat3_mul(Lr, KF, N);
    double sig[6] = {-30e3 + 2e3 * rnd(), -28e3 + 2e3 * rnd(), -33e3 + 2e3 * rnd(), 3e3 * rnd(), 3e3 * rnd(),
                     3e3 * rnd()};
    const double pc = plastic ? -31e3 : -60e3;
    const double Srs = 19e3 * (1.0 + 0.1 * rnd());
    const double w = 0.009 * (1.0 + 0.1 * rnd());
    const double dt = p->dt;
    // weights of the test functional, each term scaled to O(1) so that the
    // central differences are not swamped by rounding
    TailFwd F0;
    tail_forward(P, K, N, sig, pc, Srs, w, dt, F0);
    double mM = 0.0, mS = 0.0;
    for (int k = 0; k < 9; ++k) mM = fmax(mM, fabs(F0.M[k]));
    for (int k = 0; k < 6; ++k) mS = fmax(mS, fabs(F0.sg[k]));
    double R[9], Rs[6];
    for (int k = 0; k < 9; ++k) R[k] = rnd() / mM;
    for (int k = 0; k < 6; ++k) Rs[k] = rnd() / mS;
    const double Rp = rnd() / fabs(F0.pc);
    auto J = [&](const DevParams& PP, const double* K_, const double* N_, const double* sg_, double pc_, double Srs_,
                 double w_, int* br) {
      TailFwd F;
      tail_forward(PP, K_, N_, sg_, pc_, Srs_, w_, dt, F);
      *br = F.branch;
      double v = Rp * F.pc;
      for (int k = 0; k < 9; ++k) v += R[k] * F.M[k];
      for (int k = 0; k < 6; ++k) v += Rs[k] * F.sg[k];
      return v;
    };
    TailFwd F;
    tail_forward(P, K, N, sig, pc, Srs, w, dt, F);
    if (F.branch < 0) return ULPPM_E_NOCONV;
    if (F.branch > 0) ++npl;
    double Kb[6], Nb[9], sigb[6] = {0, 0, 0, 0, 0, 0}, pcb = 0, Srsb = 0, wb = 0, thb[4] = {0, 0, 0, 0};
    tail_reverse(P, K, N, sig, pc, Srs, w, dt, F, R, Rs, Rp, Kb, Nb, sigb, &pcb, &Srsb, &wb, thb);
    // finite differences, input by input
    auto check = [&](double analytic, double fd) {
      const double scale = fabs(analytic) + fabs(fd) + 1e-300;
      const double e = fabs(analytic - fd) / scale;
      return e;
    };
    double gmax = 0.0, emax = 0.0;
    auto fd = [&](double& x, double scale) -> double {
      const double h = 1e-6 * scale;
      const double x0 = x;
      int b1, b2;
      x = x0 + h;
      const double jp = J(P, K, N, sig, pc, Srs, w, &b1);
      x = x0 - h;
      const double jm = J(P, K, N, sig, pc, Srs, w, &b2);
      x = x0;
      if (b1 != F.branch || b2 != F.branch) return (double)NAN;
      return (jp - jm) / (2 * h);
    };
    double grads[40], fds[40];
    int ng = 0;
    double sK = 0.0, sN = 0.0, sS = 0.0;       // step sizes scaled by each input group
    for (int k = 0; k < 6; ++k) sK = fmax(sK, fabs(K[k]));
    for (int k = 0; k < 9; ++k) sN = fmax(sN, fabs(N[k]));
    for (int k = 0; k < 6; ++k) sS = fmax(sS, fabs(sig[k]));
    for (int k = 0; k < 6; ++k) { grads[ng] = Kb[k]; fds[ng++] = fd(K[k], sK); }
    for (int k = 0; k < 9; ++k) { grads[ng] = Nb[k]; fds[ng++] = fd(N[k], sN); }
    for (int k = 0; k < 6; ++k) { grads[ng] = sigb[k]; fds[ng++] = fd(sig[k], sS); }
    double pcv = pc, Srsv = Srs, wv = w;
    {
      const double h = 1e-6 * fabs(pcv);
      int b1, b2;
      const double jp = J(P, K, N, sig, pcv + h, Srs, w, &b1), jm = J(P, K, N, sig, pcv - h, Srs, w, &b2);
      grads[ng] = pcb; fds[ng++] = (b1 == F.branch && b2 == F.branch) ? (jp - jm) / (2 * h) : (double)NAN;
    }
    {
      const double h = 1e-6 * Srsv;
      int b1, b2;
      const double jp = J(P, K, N, sig, pc, Srsv + h, w, &b1), jm = J(P, K, N, sig, pc, Srsv - h, w, &b2);
      grads[ng] = Srsb; fds[ng++] = (b1 == F.branch && b2 == F.branch) ? (jp - jm) / (2 * h) : (double)NAN;
    }
    {
      const double h = 1e-6 * wv;
      int b1, b2;
      const double jp = J(P, K, N, sig, pc, Srs, wv + h, &b1), jm = J(P, K, N, sig, pc, Srs, wv - h, &b2);
      grads[ng] = wb; fds[ng++] = (b1 == F.branch && b2 == F.branch) ? (jp - jm) / (2 * h) : (double)NAN;
    }
    double* th[4] = {&P.M, &P.lam, &P.kap, &P.eta};
    for (int k = 0; k < 4; ++k) {
      double& x = *th[k];
      const double x0 = x, h = 1e-5 * fabs(x0);
      int b1, b2;
      x = x0 + h;
      P.iM2 = 1.0 / (P.M * P.M);
      const double jp = J(P, K, N, sig, pc, Srs, w, &b1);
      x = x0 - h;
      P.iM2 = 1.0 / (P.M * P.M);
      const double jm = J(P, K, N, sig, pc, Srs, w, &b2);
      x = x0;
      P.iM2 = 1.0 / (P.M * P.M);
      grads[ng] = thb[k];
      fds[ng++] = (b1 == F.branch && b2 == F.branch) ? (jp - jm) / (2 * h) : (double)NAN;
    }
    for (int k = 0; k < ng; ++k) gmax = fmax(gmax, fabs(grads[k]) * 1.0);
    // weight each input's error by its own scale times the input size so that
    // gradients that are exactly zero in one branch do not dominate
    for (int k = 0; k < ng; ++k) {
      if (std::isnan(fds[k])) continue;
      const double e = check(grads[k], fds[k]);
      if (fabs(grads[k]) + fabs(fds[k]) > 1e-9 * gmax) emax = fmax(emax, e);
#ifdef ULPPM_SELFCHECK_VERBOSE
      if (e > 1e-5) printf("case %d branch %d input %d: reverse %.10e fd %.10e\n", cs, F.branch, k, grads[k], fds[k]);
#endif
    }
    worst = fmax(worst, emax);
  }
  *max_rel = worst;
  *n_plastic = npl;
  return ULPPM_OK;
}

}  // extern "C"

namespace {

// Capacities of a context for n points and max_family members per family.
// Returns false where a bond or candidate slot would not fit an int32.
bool size_context(ulppm_ctx* ctx, int64_t n_points, int max_family) {
  ctx->cap_n = n_points;
  ctx->max_f = max_family;
  ctx->max_cells = n_points * 2 + 4096;
  ctx->bond_cap = n_points * (int64_t)max_family;
  ctx->max_c = ((max_family * 3 / 2) + 63) / 64 * 64;
  ctx->part_cap = kPartGather + 3 * 4096 + 64;
  ctx->scan_cap = (std::max<int64_t>(n_points + 1, ctx->max_cells) + kScanChunk - 1) / kScanChunk + 1;
  return ctx->bond_cap <= 2147483647LL && n_points * (int64_t)ctx->max_c <= 2147483647LL;
}

// Every scratch buffer of a context, in order: A(&pointer, bytes) places it
// (hipMalloc for ulppm_create, slices of the static array for
// ulppm_forces_static).
template <class Alloc>
void context_buffers(ulppm_ctx* ctx, Alloc&& A) {
  const int64_t n = ctx->cap_n;
  A((void**)&ctx->x, sizeof(double) * 3 * n);
  A((void**)&ctx->vh, sizeof(double) * 3 * n);
  A((void**)&ctx->vol_n, sizeof(double) * n);
  A((void**)&ctx->pscr, sizeof(double) * 12 * n);
  A((void**)&ctx->pk, sizeof(double) * 2 * n);
  A((void**)&ctx->xv, sizeof(double) * 8 * n);
  A((void**)&ctx->fown, sizeof(double) * 3 * n);
  A((void**)&ctx->cellid, sizeof(int32_t) * n);
  A((void**)&ctx->cnt, sizeof(int32_t) * n);
  A((void**)&ctx->row, sizeof(int64_t) * (n + 1));
  A((void**)&ctx->cand, sizeof(int32_t) * n * ctx->max_c);
  A((void**)&ctx->ccnt, sizeof(int32_t) * n);
  A((void**)&ctx->crev, sizeof(int32_t) * n * ctx->max_c);
  A((void**)&ctx->fbits, sizeof(unsigned long long) * n * (ctx->max_c / 64));
  A((void**)&ctx->xref, sizeof(double) * 3 * n);
  A((void**)&ctx->gate, sizeof(int32_t));
  A((void**)&ctx->ccount, sizeof(int32_t) * ctx->max_cells);
  A((void**)&ctx->ccursor, sizeof(int32_t) * ctx->max_cells);
  A((void**)&ctx->cstart, sizeof(int64_t) * (ctx->max_cells + 1));
  A((void**)&ctx->cpts, sizeof(int32_t) * n);
  A((void**)&ctx->col, sizeof(int32_t) * ctx->bond_cap);
  A((void**)&ctx->rev, sizeof(int32_t) * ctx->bond_cap);
  A((void**)&ctx->T, sizeof(double) * 4 * ctx->bond_cap);
  A((void**)&ctx->part, sizeof(double) * ctx->part_cap);
  A((void**)&ctx->scan_bsum, sizeof(int64_t) * ctx->scan_cap);
  A((void**)&ctx->grid, sizeof(Grid));
  A((void**)&ctx->ctr, sizeof(unsigned long long) * C_NCOUNT * kStripes);
  A((void**)&ctx->ctr_sum, sizeof(unsigned long long) * C_NCOUNT);
  A((void**)&ctx->E, sizeof(double) * 3);
}

// The bond kernel's dynamic LDS may exceed the default cap for large max_family.
void set_bond_lds_limits(int max_family) {
  const int l64 = (int)bond_lds(max_family, false, kBondThreads),
            l32 = (int)bond_lds(max_family, true, kBondThreads);
  bond_lds_limit<double, false, false>(l64);
  bond_lds_limit<double, false, true>(l64);
  bond_lds_limit<double, true, false>(l64);
  bond_lds_limit<double, true, true>(l64);
  bond_lds_limit<float, false, false>(l32);
  bond_lds_limit<float, false, true>(l32);
  bond_lds_limit<float, true, false>(l32);
  bond_lds_limit<float, true, true>(l32);
}

}  // namespace

extern "C" {

int ulppm_create(ulppm_ctx** out, int64_t n_points, int32_t max_family, void* hip_stream) {
  ulppm_ctx* ctx = nullptr;
  if (!out) return ULPPM_E_ARG;
  *out = nullptr;
  if (n_points <= 0 || n_points > 2147483647LL) return ULPPM_E_ARG;
  if (max_family == 0) max_family = 152;
  if (max_family < 8 || max_family > 1024) return ULPPM_E_ARG;
  ctx = new ulppm_ctx();
  ctx->stream = (hipStream_t)hip_stream;
  if (!size_context(ctx, n_points, max_family)) {
    delete ctx;
    return ULPPM_E_ARG;   // bond slots are int32
  }
  hipError_t e = hipSuccess;
  context_buffers(ctx, [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes > 0 ? bytes : 8);
  });
  if (e != hipSuccess) {
    ulppm_destroy(ctx);
    return ULPPM_E_HIP;
  }
  k_fill<double><<<1, 64, 0, ctx->stream>>>(ctx->E, 3, 0.0);
  ctx->have_events = true;
  for (int k = 0; k < kTimedSteps && ctx->have_events; ++k)
    for (int ph = 0; ph < kPhases; ++ph)
      for (int b = 0; b < 2; ++b)
        if (hipEventCreate(&ctx->ev[k][ph][b]) != hipSuccess) ctx->have_events = false;
  if (!ctx->have_events) {
    ulppm_destroy(ctx);
    return ULPPM_E_HIP;
  }
  set_bond_lds_limits(max_family);
  if (hipGetLastError() != hipSuccess) {
    ulppm_destroy(ctx);
    return ULPPM_E_HIP;
  }
  *out = ctx;
  return ULPPM_OK;
}

int ulppm_destroy(ulppm_ctx* ctx) {
  if (!ctx) return ULPPM_E_ARG;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  void* ptrs[] = {ctx->x, ctx->vh, ctx->vol_n, ctx->pscr, ctx->pk, ctx->xv, ctx->fown, ctx->cellid, ctx->cnt, ctx->row, ctx->cand,
                  ctx->ccnt, ctx->crev, ctx->fbits, ctx->xref, ctx->gate,
                  ctx->ccount, ctx->ccursor, ctx->cstart, ctx->cpts, ctx->col, ctx->rev, ctx->T,
                  ctx->part, ctx->scan_bsum, ctx->grid, ctx->ctr, ctx->ctr_sum, ctx->E, ctx->adj,
                  ctx->adj_slot, ctx->adj_hist, ctx->hist[0], ctx->hist[1], ctx->hist_row, ctx->hist_col,
                  ctx->hist_map};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (ctx->have_events)
    for (int k = 0; k < kTimedSteps; ++k)
      for (int ph = 0; ph < kPhases; ++ph)
        for (int b = 0; b < 2; ++b)
          if (ctx->ev[k][ph][b]) (void)hipEventDestroy(ctx->ev[k][ph][b]);
  delete ctx;
  return ULPPM_OK;
}

const char* ulppm_last_error(const ulppm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "NULL context";
}

int ulppm_reset_energy(ulppm_ctx* ctx) {
  if (!ctx) return ULPPM_E_ARG;
  k_fill<double><<<1, 64, 0, ctx->stream>>>(ctx->E, 3, 0.0);
  HIPCHK(hipGetLastError());
  return ULPPM_OK;
}

int ulppm_build_families(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_params* p, int64_t* row_ptr,
                         int32_t* col, int64_t col_cap, int64_t* n_bonds_out) {
  if (!ctx) return ULPPM_E_ARG;
  int rc = check_state(ctx, S);
  if (rc) return rc;
  if (!p || !(p->delta > 0.0)) return fail(ctx, ULPPM_E_ARG, "delta must be > 0");
  const int64_t n = S->n;
  if ((rc = zero_counters(ctx))) return rc;
  k_positions<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(*S, ctx->x, ctx->vh, ctx->vol_n);
  HIPCHK(hipGetLastError());
  if ((rc = build_families(ctx, n, p->delta, true))) return rc;
  if ((rc = read_counters(ctx))) return rc;
  if ((rc = counters_to_status(ctx))) return rc;
  int64_t nb = 0;
  HIPCHK(hipMemcpyAsync(&nb, ctx->row + n, sizeof(nb), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (n_bonds_out) *n_bonds_out = nb;
  if (row_ptr) {
    k_export_rows<<<blocks_for(n + 1, 256), 256, 0, ctx->stream>>>(n, ctx->row, row_ptr);
    HIPCHK(hipGetLastError());
  }
  if (col) {
    if (col_cap < nb) return fail(ctx, ULPPM_E_CAPACITY, "col_cap smaller than the bond count");
    k_copy_i32<<<blocks_for(nb, 256), 256, 0, ctx->stream>>>(ctx->col, col, nb);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ULPPM_OK;
}

}  // extern "C"

namespace {

// Algorithm 1 alone at the current state (ulppm_forces, ulppm_forces_static).
int forces_impl(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_params* p, double dt_inc, double* f[3],
                double* T_out[3], ulppm_report* rep) {
  int rc = check_state(ctx, S);
  if (rc) return rc;
  if ((rc = check_params(ctx, p))) return rc;
  if (!f || !f[0] || !f[1] || !f[2]) return fail(ctx, ULPPM_E_ARG, "f is NULL");
  if (!(dt_inc >= 0.0) || !std::isfinite(dt_inc)) return fail(ctx, ULPPM_E_ARG, "dt_inc must be finite and >= 0");
  const int64_t n = S->n;
  if ((rc = zero_counters(ctx))) return rc;
  k_positions<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(*S, ctx->x, ctx->vh, ctx->vol_n);
  HIPCHK(hipGetLastError());
  if ((rc = build_families(ctx, n, p->delta, true))) return rc;
  if ((rc = bond_pass(ctx, S, p, dt_inc, false))) return rc;
  if ((rc = gather_pass(ctx, S, p, G_FORCES, ctx->pscr + 4 * n, f))) return rc;
  if ((rc = read_counters(ctx))) return rc;
  fill_report(ctx, n, rep, 0);
  if ((rc = counters_to_status(ctx))) return rc;
  if (T_out) {
    int64_t nb = 0;
    HIPCHK(hipMemcpyAsync(&nb, ctx->row + n, sizeof(nb), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const bool mixed = p->precision == ULPPM_MIXED;
    for (int c = 0; c < 3; ++c)
      if (T_out[c]) {
        if (mixed)
          k_unpack_T<float><<<blocks_for(nb, 256), 256, 0, ctx->stream>>>(
              reinterpret_cast<const Quad<float>*>(ctx->T), c, T_out[c], nb);
        else if (own_sums(ctx, p))
          k_unpack_T_scaled<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(
              reinterpret_cast<const Quad<double>*>(ctx->T), c, ctx->row, ctx->vol_n, n, T_out[c]);
        else
          k_unpack_T<double><<<blocks_for(nb, 256), 256, 0, ctx->stream>>>(
              reinterpret_cast<const Quad<double>*>(ctx->T), c, T_out[c], nb);
      }
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ULPPM_OK;
}

// Scratch of ulppm_forces_static: one file-scope array per device, holding
// the buffers of a context for kStaticPoints points and kStaticFamily
// members per family.  Host code never uses the array's name (a host-side
// stand-in); it uses the device address hipGetSymbolAddress returns.
constexpr int64_t kStaticPoints = ULPPM_STATIC_MAX_POINTS;
constexpr int kStaticFamily = ULPPM_STATIC_MAX_FAMILY;
constexpr size_t kStaticAlign = 256;
constexpr size_t kStaticBytes = 16u << 20;   // 16 MiB (about 14 MiB used); checked against the buffer list at set-up
constexpr int kStaticDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

struct StaticSlot {
  ulppm_ctx ctx;          // buffers sliced from this device's scratch array
  bool ready = false;
};
StaticSlot g_static[kStaticDevices];
std::mutex g_static_mu;

// Set-up on the current device, once: the array's device address, the
// context's buffers sliced from it (256-byte aligned), the bond kernel's LDS
// limits and zeroed energies.  Returns the context or null (code in *rc).
ulppm_ctx* static_context(hipStream_t stream, int* rc) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kStaticDevices) {
    *rc = dev >= kStaticDevices ? ULPPM_E_ARG : ULPPM_E_HIP;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticSlot& sl = g_static[dev];
  ulppm_ctx* ctx = &sl.ctx;
  if (!sl.ready) {
    unsigned char* base = nullptr;
    if (hipGetSymbolAddress((void**)&base, HIP_SYMBOL(scratch)) != hipSuccess || !base) {
      *rc = ULPPM_E_HIP;
      return nullptr;
    }
    if (!size_context(ctx, kStaticPoints, kStaticFamily)) {
      *rc = ULPPM_E_ARG;
      return nullptr;
    }
    size_t off = 0;
    bool fits = true;
    context_buffers(ctx, [&](void** p, size_t bytes) {
      off = (off + kStaticAlign - 1) / kStaticAlign * kStaticAlign;
      if (off + bytes > kStaticBytes) fits = false;
      *p = fits ? (void*)(base + off) : nullptr;
      off += bytes;
    });
    if (!fits) {
      *rc = ULPPM_E_HIP;      // the array is smaller than the buffer list: a build error
      return nullptr;
    }
    ctx->have_events = false;
    set_bond_lds_limits(kStaticFamily);
    k_fill<double><<<1, 64, 0, stream>>>(ctx->E, 3, 0.0);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) {
      *rc = ULPPM_E_HIP;
      return nullptr;
    }
    sl.ready = true;
  }
  ctx->stream = stream;
  ctx->contact = ContactDev{};
  ctx->hist_n = 0;
  *rc = ULPPM_OK;
  return ctx;
}

}  // namespace

extern "C" {

int ulppm_forces(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_params* p, double dt_inc, double* f[3],
                 double* T_out[3], ulppm_report* rep) {
  if (!ctx) return ULPPM_E_ARG;
  return forces_impl(ctx, S, p, dt_inc, f, T_out, rep);
}

int ulppm_forces_static(const ulppm_state* S, const ulppm_params* p, double dt_inc, double* f[3],
                        double* T_out[3], ulppm_report* rep, void* hip_stream) {
  if (!S || S->n <= 0 || S->n > kStaticPoints) return ULPPM_E_ARG;
  int rc = ULPPM_OK;
  ulppm_ctx* ctx = static_context((hipStream_t)hip_stream, &rc);
  if (!ctx) return rc;
  return forces_impl(ctx, S, p, dt_inc, f, T_out, rep);
}

int ulppm_init_state(ulppm_ctx* ctx, ulppm_state* S, const ulppm_params* p, double ocr) {
  if (!ctx) return ULPPM_E_ARG;
  int rc = check_state(ctx, S);
  if (rc) return rc;
  if ((rc = check_params(ctx, p))) return rc;
  if (!(ocr >= 1.0)) return fail(ctx, ULPPM_E_ARG, "ocr must be >= 1");
  const int64_t n = S->n;
  ctx->hist_n = 0;                        // a new state: no bond history yet
  if ((rc = zero_counters(ctx))) return rc;
  DevParams P = dev_params(p);
  k_init_points<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(*S, P, ocr);
  k_positions<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(*S, ctx->x, ctx->vh, ctx->vol_n);
  HIPCHK(hipGetLastError());
  if ((rc = build_families(ctx, n, p->delta, true))) return rc;
  if ((rc = bond_pass(ctx, S, p, 0.0, false))) return rc;
  if ((rc = gather_pass(ctx, S, p, G_INIT, S->mass, nullptr))) return rc;
  k_fill<double><<<1, 64, 0, ctx->stream>>>(ctx->E, 3, 0.0);
  HIPCHK(hipGetLastError());
  if ((rc = read_counters(ctx))) return rc;
  return counters_to_status(ctx);
}

int ulppm_dt_crit(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_params* p, double* dt_out) {
  if (!ctx) return ULPPM_E_ARG;
  int rc = check_state(ctx, S);
  if (rc) return rc;
  if ((rc = check_params(ctx, p))) return rc;
  if (!dt_out) return fail(ctx, ULPPM_E_ARG, "dt_out is NULL");
  const int64_t n = S->n;
  if ((rc = zero_counters(ctx))) return rc;
  k_positions<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(*S, ctx->x, ctx->vh, ctx->vol_n);
  HIPCHK(hipGetLastError());
  if ((rc = build_families(ctx, n, p->delta, true))) return rc;
  const int nb = blocks_for(n, 256, 1024);
  // bond micromodulus: 3D, or plane strain per unit thickness (Poisson 1/4)
  const double C = p->plane ? 72.0 * p->K / (5.0 * M_PI * std::pow(p->delta, 3))
                            : 18.0 * p->K / (M_PI * std::pow(p->delta, 4));
  k_dtcrit<<<nb, 256, 0, ctx->stream>>>(n, ctx->row, ctx->col, ctx->x, S->vol, S->phi, C, p->rho_s,
                                         ctx->part + kPartRed);
  HIPCHK(hipGetLastError());
  double h[1024];
  HIPCHK(hipMemcpyAsync(h, ctx->part + kPartRed, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
  if ((rc = read_counters(ctx))) return rc;
  if ((rc = counters_to_status(ctx))) return rc;
  double best = INFINITY;
  for (int b = 0; b < nb; ++b) best = std::fmin(best, h[b]);
  *dt_out = best;
  return ULPPM_OK;
}

constexpr size_t kMaxLds = 160 * 1024 - 1024;   // dynamic LDS of one workgroup (CDNA4: 160 KB per CU)

size_t adj_lds(int max_f) {
  return (size_t)max_f * (3 * sizeof(Quad<double>) + sizeof(MRec<double>) + 16 * sizeof(double) +
                          (size_t)((max_f + 63) / 64) * sizeof(unsigned long long));
}

int ulppm_set_contact(ulppm_ctx* ctx, const ulppm_contact* c) {
  if (!ctx) return ULPPM_E_ARG;
  if (!c || !(c->cs > 0.0)) {
    ctx->contact = ContactDev{};
    return ULPPM_OK;
  }
  if (!(c->spacing > 0.0) || !(c->delta_c > 0.0) || !(c->mu_f >= 0.0) || !std::isfinite(c->cs) ||
      !std::isfinite(c->origin[0]) || !std::isfinite(c->origin[1]) || !std::isfinite(c->origin[2]))
    return fail(ctx, ULPPM_E_ARG, "contact: spacing and delta_c must be > 0, mu_f >= 0, values finite");
  if (c->n[0] < 1 || c->n[1] < 1 || c->n[2] < 1 || (int64_t)c->n[0] * c->n[1] * c->n[2] > 2147483647LL)
    return fail(ctx, ULPPM_E_ARG, "contact: site counts must be >= 1 with at most 2^31-1 sites");
  ContactDev d;
  d.cs = c->cs;
  d.mu_f = c->mu_f;
  d.dc = c->delta_c;
  d.dc2 = c->delta_c * c->delta_c;
  d.ox = c->origin[0];
  d.oy = c->origin[1];
  d.oz = c->origin[2];
  d.h = c->spacing;
  d.Vs = c->spacing * c->spacing * c->spacing;
  d.nx = c->n[0];
  d.ny = c->n[1];
  d.nz = c->n[2];
  d.on = 1;
  ctx->contact = d;
  return ULPPM_OK;
}

// Scratch of the bond-history adjoint, once both the adjoint scratch and the
// bond states are reserved (whichever reservation comes second allocates it).
static int reserve_adj_hist(ulppm_ctx* ctx) {
  if (ctx->adj_hist || !ctx->adj || !ctx->hist[0]) return ULPPM_OK;
  const hipError_t e = hipMalloc((void**)&ctx->adj_hist, sizeof(double) * 16 * (size_t)ctx->bond_cap);
  if (e != hipSuccess) {
    ctx->adj_hist = nullptr;
    return fail(ctx, ULPPM_E_HIP, std::string("bond-history adjoint scratch: ") + hipGetErrorString(e));
  }
  return ULPPM_OK;
}

int ulppm_history_reserve(ulppm_ctx* ctx) {
  if (!ctx) return ULPPM_E_ARG;
  if (ctx->hist[0]) return ULPPM_OK;
  const size_t st = sizeof(double) * 8 * (size_t)ctx->bond_cap;
  void* a = nullptr;
  void* b = nullptr;
  void* r = nullptr;
  void* c = nullptr;
  void* m = nullptr;
  hipError_t e = hipMalloc(&a, st);
  if (e == hipSuccess) e = hipMalloc(&b, st);
  if (e == hipSuccess) e = hipMalloc(&r, sizeof(int64_t) * (size_t)(ctx->cap_n + 1));
  if (e == hipSuccess) e = hipMalloc(&c, sizeof(int32_t) * (size_t)ctx->bond_cap);
  if (e == hipSuccess) e = hipMalloc(&m, sizeof(int64_t) * (size_t)ctx->bond_cap);
  if (e != hipSuccess) {
    for (void* q : {a, b, r, c, m})
      if (q) (void)hipFree(q);
    return fail(ctx, ULPPM_E_HIP, std::string("bond history: ") + hipGetErrorString(e));
  }
  ctx->hist[0] = static_cast<double*>(a);
  ctx->hist[1] = static_cast<double*>(b);
  ctx->hist_row = static_cast<int64_t*>(r);
  ctx->hist_col = static_cast<int32_t*>(c);
  ctx->hist_map = static_cast<int64_t*>(m);
  ctx->hist_last = 0;
  ctx->hist_n = 0;
  return reserve_adj_hist(ctx);
}

int ulppm_history_export(ulppm_ctx* ctx, int64_t* row_out, int32_t* col_out, double* st_out, int64_t cap,
                         int64_t* nb_out) {
  if (!ctx) return ULPPM_E_ARG;
  if (!nb_out) return fail(ctx, ULPPM_E_ARG, "nb_out is NULL");
  if (!ctx->hist[0] || ctx->hist_n == 0) return fail(ctx, ULPPM_E_ARG, "no bond history is held");
  const int64_t n = ctx->hist_n;
  int64_t nb = 0;
  HIPCHK(hipMemcpyAsync(&nb, ctx->hist_row + n, sizeof(nb), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *nb_out = nb;
  if (!row_out && !col_out && !st_out) return ULPPM_OK;
  if (cap < nb) return fail(ctx, ULPPM_E_CAPACITY, "cap is smaller than the bond count");
  if (row_out)
    HIPCHK(hipMemcpyAsync(row_out, ctx->hist_row, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, ctx->stream));
  if (col_out)
    HIPCHK(hipMemcpyAsync(col_out, ctx->hist_col, sizeof(int32_t) * nb, hipMemcpyDeviceToDevice, ctx->stream));
  if (st_out)
    HIPCHK(hipMemcpyAsync(st_out, ctx->hist[ctx->hist_last], sizeof(double) * 8 * nb, hipMemcpyDeviceToDevice,
                          ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ULPPM_OK;
}

int ulppm_history_import(ulppm_ctx* ctx, int64_t n, const int64_t* row, const int32_t* col, const double* st,
                         int64_t n_bonds) {
  if (!ctx) return ULPPM_E_ARG;
  if (!ctx->hist[0]) return fail(ctx, ULPPM_E_ARG, "call ulppm_history_reserve first");
  if (n < 1 || n > ctx->cap_n) return fail(ctx, ULPPM_E_ARG, "n out of range");
  if (n_bonds < 0 || n_bonds > ctx->bond_cap) return fail(ctx, ULPPM_E_ARG, "n_bonds out of range");
  if (n_bonds == 0) {
    ctx->hist_n = 0;                               // none held: every bond starts from its point
    return ULPPM_OK;
  }
  if (!row || !col || !st) return fail(ctx, ULPPM_E_ARG, "row, col and st are needed when n_bonds > 0");
  HIPCHK(hipMemcpyAsync(ctx->hist_row, row, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->hist_col, col, sizeof(int32_t) * n_bonds, hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->hist[ctx->hist_last], st, sizeof(double) * 8 * n_bonds, hipMemcpyDeviceToDevice,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->hist_n = n;
  return ULPPM_OK;
}

int ulppm_adjoint_reserve(ulppm_ctx* ctx) {
  if (!ctx) return ULPPM_E_ARG;
  if (ctx->adj) return ULPPM_OK;
  const int64_t n = ctx->cap_n;
  const size_t pts = sizeof(double) * (size_t)(45 * n + 4 * (n + 8));
  HIPCHK(hipMalloc((void**)&ctx->adj, pts));
  // per bond slot: the adjoint contributions (x 3, v_half 3, V 1) and the
  // bond tail's forward solution (8)
  const hipError_t e = hipMalloc((void**)&ctx->adj_slot, sizeof(double) * 16 * (size_t)ctx->bond_cap);
  if (e != hipSuccess) {
    (void)hipFree(ctx->adj);
    ctx->adj = nullptr;
    return fail(ctx, ULPPM_E_HIP, std::string("adjoint scratch: ") + hipGetErrorString(e));
  }
  for (const void* k : {(const void*)k_adj_bond<false, double, false>, (const void*)k_adj_bond<true, double, false>,
                        (const void*)k_adj_bond<false, float, false>, (const void*)k_adj_bond<true, float, false>,
                        (const void*)k_adj_bond<false, double, true>, (const void*)k_adj_bond<true, double, true>,
                        (const void*)k_adj_bond<false, float, true>, (const void*)k_adj_bond<true, float, true>})
    HIPCHK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)std::min(adj_lds(ctx->max_f), kMaxLds)));
  return reserve_adj_hist(ctx);
}

int ulppm_adjoint_init(ulppm_ctx* ctx, const ulppm_state* S0, const ulppm_params* p, double ocr,
                       const ulppm_state* adj0, double* s_bar, double* theta_bar) {
  if (!ctx) return ULPPM_E_ARG;
  int rc = check_state(ctx, S0);
  if (rc) return rc;
  if ((rc = check_state(ctx, adj0))) return rc;
  if ((rc = check_params(ctx, p))) return rc;
  if (!s_bar || !theta_bar) return fail(ctx, ULPPM_E_ARG, "s_bar or theta_bar is NULL");
  if (!ctx->adj) return fail(ctx, ULPPM_E_ARG, "call ulppm_adjoint_reserve first");
  if (!(ocr >= 1.0)) return fail(ctx, ULPPM_E_ARG, "ocr must be >= 1");
  const int64_t n = S0->n;
  if (adj0->n != n) return fail(ctx, ULPPM_E_ARG, "adjoint state must match the state size");
  const int nb = blocks_for(n, 256, 2048);
  double* part = ctx->adj + 45 * n;     // 4 (n + 8) doubles, nb <= n + 8
  k_adj_init<<<nb, 256, 0, ctx->stream>>>(*S0, *adj0, dev_params(p), ocr, s_bar, part);
  k_adj_theta<<<1, kThetaThreads, 0, ctx->stream>>>(part, (int64_t)nb, theta_bar);
  HIPCHK(hipGetLastError());
  return ULPPM_OK;
}

// Forward re-run of step n -> n+1 on a scratch copy F of state n (in the
// adjoint scratch), leaving x^{n+1}, v_half, V^n, the families and F =
// state n+1 in the context.
static int adjoint_rerun(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_params* p, const DevParams& P,
                         ulppm_state& F) {
  const int64_t n = S->n;
  double* q = ctx->adj;
  int rc;
  for (int c = 0; c < 3; ++c) {
    F.u[c] = q + (0 + c) * n;
    F.uc[c] = q + (3 + c) * n;
    F.v[c] = q + (6 + c) * n;
    F.a[c] = q + (9 + c) * n;
  }
  F.vol = q + 12 * n; F.phi = q + 13 * n; F.J = q + 14 * n; F.Sr = q + 15 * n; F.mass = q + 16 * n;
  for (int k = 0; k < 6; ++k) F.sig[k] = q + (17 + k) * n;
  F.pc = q + 23 * n;
  const int cb = blocks_for(n, 256, 4096);
  for (int c = 0; c < 3; ++c) {
    k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->u[c], F.u[c], n);
    k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->uc[c], F.uc[c], n);
    k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->v[c], F.v[c], n);
    k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->a[c], F.a[c], n);
  }
  k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->vol, F.vol, n);
  k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->phi, F.phi, n);
  k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->J, F.J, n);
  k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->Sr, F.Sr, n);
  k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->mass, F.mass, n);
  for (int k = 0; k < 6; ++k) k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->sig[k], F.sig[k], n);
  k_copy_f64<<<cb, 256, 0, ctx->stream>>>(S->pc, F.pc, n);
  HIPCHK(hipGetLastError());
  const int npb = blocks_for(n, 256, 2048);
  k_predict<<<npb, 256, 0, ctx->stream>>>(F, P, ctx->x, ctx->vh, ctx->vol_n, ctx->part + kPartPred);
  HIPCHK(hipGetLastError());
  if ((rc = build_families(ctx, n, p->delta, true))) return rc;
  if ((rc = bond_pass(ctx, &F, p, p->dt, true))) return rc;
  if ((rc = gather_pass(ctx, &F, p, G_STEP, F.mass, nullptr))) return rc;
  return ULPPM_OK;
}

// Bond states of the bond-history adjoint: those after step n (in the
// order of the families row_n / col_n, none when nb_n == 0), the adjoint of
// those after step n+1 (order of the families of state n+1) and the adjoint
// of those after step n (written).
struct HistAdj {
  int64_t nb_n;
  const int64_t* row_n;
  const int32_t* col_n;
  const double* hist_n;
  const double* hist_bar1;
  double* hist_bar0;
};

static int adjoint_step_impl(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_state* S1, const ulppm_params* p,
                             const ulppm_state* adj1, ulppm_state* adj0, double* theta_bar, ulppm_report* rep,
                             const HistAdj* H) {
  if (!ctx) return ULPPM_E_ARG;
  int rc = check_state(ctx, S);
  if (rc) return rc;
  if (S1 && (rc = check_state(ctx, S1))) return rc;
  if ((rc = check_state(ctx, adj1))) return rc;
  if ((rc = check_state(ctx, adj0))) return rc;
  if ((rc = check_params(ctx, p))) return rc;
  if (!theta_bar) return fail(ctx, ULPPM_E_ARG, "theta_bar is NULL");
  if (!ctx->adj) return fail(ctx, ULPPM_E_ARG, "call ulppm_adjoint_reserve first");
  if (!H && p->history)
    return fail(ctx, ULPPM_E_ARG, "with the history on the bonds use ulppm_adjoint_step_bond_history");
  if (H) {
    if (p->history != ULPPM_HISTORY_BOND) return fail(ctx, ULPPM_E_ARG, "p->history must be ULPPM_HISTORY_BOND");
    if (!S1) return fail(ctx, ULPPM_E_ARG, "the bond-history adjoint needs state n+1");
    if (!ctx->adj_hist) return fail(ctx, ULPPM_E_ARG, "call ulppm_history_reserve and ulppm_adjoint_reserve first");
    if (!H->hist_bar1) return fail(ctx, ULPPM_E_ARG, "hist_bar_np1 is NULL");
    if (H->nb_n < 0 || H->nb_n > ctx->bond_cap) return fail(ctx, ULPPM_E_ARG, "n_bonds_n out of range");
    if (H->nb_n > 0 && (!H->row_n || !H->col_n || !H->hist_n || !H->hist_bar0))
      return fail(ctx, ULPPM_E_ARG, "row_n, col_n, hist_n and hist_bar_n are needed when n_bonds_n > 0");
  }
  if (p->force_mode != ULPPM_FORCE_CONJUGATE)
    return fail(ctx, ULPPM_E_ARG, "the adjoint supports conjugate force states");
  if (!(p->dt > 0.0)) return fail(ctx, ULPPM_E_ARG, "dt must be > 0");
  const int64_t n = S->n;
  if (adj1->n != n || adj0->n != n || (S1 && S1->n != n))
    return fail(ctx, ULPPM_E_ARG, "adjoint states must match the state size");
  if ((rc = zero_counters(ctx))) return rc;
  double* q = ctx->adj;
  DevParams P = dev_params(p);
  ulppm_state F = S1 ? *S1 : *S;
  if (S1) {
    // state n+1 given: positions, half-step velocities and families only
    k_adj_kin<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(*S, *S1, P, ctx->x, ctx->vh, ctx->vol_n);
    HIPCHK(hipGetLastError());
    // the candidate lists are rebuilt only when a point has left half the
    // skin since they were built (either direction in time)
    if ((rc = build_families(ctx, n, p->delta, false))) return rc;
  } else if ((rc = adjoint_rerun(ctx, S, p, P, F))) {
    return rc;
  }
  // reverse
  double* r = q + 24 * n;

  double* own_x = r;          // 3n
  double* own_vh = r + 3 * n; // 3n
  double* own_V = r + 6 * n;
  double* sigb = r + 7 * n;   // 6n
  double* pcb = r + 13 * n;
  double* Jb = r + 14 * n;
  double* phib = r + 15 * n;
  double* sb = r + 16 * n;
  double* fbar = r + 17 * n;  // 3n
  double* Mbt = r + 20 * n;
  double* thpart = r + 21 * n;
  k_adj_point1<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, S->fixed, F.a[0], F.a[1], F.a[2], F.mass, adj1->v[0],
                                                           adj1->v[1], adj1->v[2], adj1->a[0], adj1->a[1],
                                                           adj1->a[2], adj1->mass, 0.5 * p->dt, p->g[0], p->g[1],
                                                           p->g[2], fbar, Mbt);
  HIPCHK(hipGetLastError());
  AdjArgs A;
  A.n = n;
  A.per = (n + 7) / 8;
  A.row = ctx->row; A.col = ctx->col; A.rev = ctx->rev;
  A.x = ctx->x; A.vh = ctx->vh; A.vol_n = ctx->vol_n; A.xv = ctx->xv;
  A.J = S->J; A.phi = S->phi; A.s = S->s;
  for (int k = 0; k < 6; ++k) { A.sig[k] = S->sig[k]; A.sig1[k] = F.sig[k]; A.sigb1[k] = adj1->sig[k]; }
  A.pc = S->pc;
  A.J1 = F.J; A.phi1 = F.phi; A.Sr1 = F.Sr; A.V1 = F.vol; A.pc1 = F.pc;
  A.fbar = fbar; A.Mbt = Mbt;
  A.Vb1 = adj1->vol; A.phib1 = adj1->phi; A.Jb1 = adj1->J; A.Srb1 = adj1->Sr; A.pcb1 = adj1->pc;
  A.own_x = own_x; A.own_vh = own_vh; A.own_V = own_V; A.sigb = sigb; A.pcb = pcb; A.Jb = Jb; A.phib = phib;
  A.sb = sb;
  A.slot_x = ctx->adj_slot;
  A.slot_vh = ctx->adj_slot + 3;
  A.slot_V = ctx->adj_slot + 6;
  A.fwd = ctx->adj_slot + 8 * ctx->bond_cap;
  A.thpart = thpart;
  A.ctr = ctx->ctr;
  A.cap = ctx->bond_cap;
  A.dt = p->dt;
  // LDS for the largest family the forward calls on this context reported:
  // the step's families are those of the forward step it reverses, so no
  // wait for this step's counters is needed (a larger family would stop its
  // block and fail the step).  Without such a report, the largest family of
  // this step.
  A.max_f = ctx->seen_max_f;
  if (A.max_f <= 0 || A.max_f > ctx->max_f || adj_lds(A.max_f) > kMaxLds) {
    if ((rc = read_counters(ctx))) return rc;
    if ((rc = counters_to_status(ctx))) return rc;
    A.max_f = std::max<int>(1, (int)ctx->h_ctr[C_MAXFAM]);
  }
  const size_t lds = adj_lds(A.max_f);
  if (lds > kMaxLds)
    return fail(ctx, ULPPM_E_CAPACITY, "adjoint: a family of " + std::to_string(A.max_f) +
                                           " members exceeds the workgroup's LDS");
  const unsigned grid = (unsigned)(8 * A.per);
  const size_t carry_lds = 4 * sizeof(int32_t) * (size_t)ctx->max_f;
  const int have = H && H->nb_n > 0 ? 1 : 0;
  if (H) {
    // the start states of this step's bonds, carried from the bonds after step n
    A.hstart = ctx->adj_hist;
    A.hbar1 = H->hist_bar1;
    A.hbar0s = ctx->adj_hist + 8 * ctx->bond_cap;
    k_hist_carry<<<walk_grid(n), 256, carry_lds, ctx->stream>>>(n, ctx->row, ctx->col, H->row_n, H->col_n, have,
                                                                ctx->max_f, H->hist_n, ctx->adj_hist, *S);
    HIPCHK(hipGetLastError());
  }
  k_pack<<<blocks_for(n, 256, 8192), 256, 0, ctx->stream>>>(n, ctx->x, ctx->vh, ctx->vol_n, ctx->xv);
  const bool mixed = p->precision == ULPPM_MIXED;
  const bool lin = p->b1 == 0.0 && p->b2 == 1.0;        // Eq. 45 reduces to P = p_c
  auto go = [&](auto hist_c, auto acc_c, auto lin_c) {
    k_adj_bond<decltype(hist_c)::value, typename decltype(acc_c)::type, decltype(lin_c)::value>
        <<<grid, kBondThreads, lds, ctx->stream>>>(A, P);
  };
  using T_ = std::true_type;
  using F_ = std::false_type;
  using D_ = std::common_type<double>;
  using S_ = std::common_type<float>;
  if (H && mixed) lin ? go(T_{}, S_{}, T_{}) : go(T_{}, S_{}, F_{});
  else if (H) lin ? go(T_{}, D_{}, T_{}) : go(T_{}, D_{}, F_{});
  else if (mixed) lin ? go(F_{}, S_{}, T_{}) : go(F_{}, S_{}, F_{});
  else lin ? go(F_{}, D_{}, T_{}) : go(F_{}, D_{}, F_{});
  HIPCHK(hipGetLastError());
  if (H) {
    if (have) {
      const int64_t len = 8 * H->nb_n;
      k_fill<double><<<blocks_for(len, 256, 4096), 256, 0, ctx->stream>>>(H->hist_bar0, len, 0.0);
    }
    k_adj_hist_carry<<<walk_grid(n), 256, carry_lds, ctx->stream>>>(n, ctx->row, ctx->col, H->row_n, H->col_n,
                                                                    have, ctx->max_f, A.hbar0s, H->hist_bar0, sigb,
                                                                    pcb);
    HIPCHK(hipGetLastError());
  }
  k_adj_point2<<<walk_grid(n), 256, 0, ctx->stream>>>(n, ctx->row, ctx->rev, S->fixed, own_x, own_vh, own_V,
                                                      A.slot_x, A.slot_vh, A.slot_V, ctx->bond_cap, sigb, pcb, Jb,
                                                      phib, sb, *adj1, *adj0, p->dt, ctx->contact, p->plane != 0, fbar, ctx->x,
                                                      ctx->vh, ctx->vol_n);
  k_adj_theta<<<1, kThetaThreads, 0, ctx->stream>>>(thpart, (int64_t)grid, theta_bar);
  HIPCHK(hipGetLastError());
  if ((rc = read_counters(ctx))) return rc;
  fill_report(ctx, n, rep, 1);
  return counters_to_status(ctx);
}

int ulppm_adjoint_step(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_state* S1, const ulppm_params* p,
                       const ulppm_state* adj1, ulppm_state* adj0, double* theta_bar, ulppm_report* rep) {
  return adjoint_step_impl(ctx, S, S1, p, adj1, adj0, theta_bar, rep, nullptr);
}

int ulppm_adjoint_step_bond_history(ulppm_ctx* ctx, const ulppm_state* S, const ulppm_state* S1,
                                    const ulppm_params* p, int64_t n_bonds_n, const int64_t* row_n,
                                    const int32_t* col_n, const double* hist_n, const double* hist_bar_np1,
                                    const ulppm_state* adj1, ulppm_state* adj0, double* hist_bar_n,
                                    double* theta_bar, ulppm_report* rep) {
  const HistAdj H{n_bonds_n, row_n, col_n, hist_n, hist_bar_np1, hist_bar_n};
  return adjoint_step_impl(ctx, S, S1, p, adj1, adj0, theta_bar, rep, &H);
}

int ulppm_step(ulppm_ctx* ctx, ulppm_state* S, const ulppm_params* p, int32_t n_steps, ulppm_report* rep) {
  if (!ctx) return ULPPM_E_ARG;
  int rc = check_state(ctx, S);
  if (rc) return rc;
  if ((rc = check_params(ctx, p))) return rc;
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(ctx, ULPPM_E_ARG, "dt must be > 0");
  if (n_steps < 0) return fail(ctx, ULPPM_E_ARG, "n_steps < 0");
  const int64_t n = S->n;
  if ((rc = zero_counters(ctx))) return rc;
  DevParams P = dev_params(p);
  const int npb = blocks_for(n, 256, 2048);
  const int64_t timed = p->timing ? std::min<int64_t>(n_steps, kTimedSteps) : 0;
  const bool bond_history = p->history == ULPPM_HISTORY_BOND;
  if (bond_history && !ctx->hist[0]) return fail(ctx, ULPPM_E_ARG, "call ulppm_history_reserve first");
  auto mark = [&](int64_t k, int ph, int b) {
    if (k < timed) (void)hipEventRecord(ctx->ev[k][ph][b], ctx->stream);
  };
  for (int32_t k = 0; k < n_steps; ++k) {
    mark(k, 0, 0);
    k_predict<<<npb, 256, 0, ctx->stream>>>(*S, P, ctx->x, ctx->vh, ctx->vol_n, ctx->part + kPartPred);
    HIPCHK(hipGetLastError());
    mark(k, 0, 1);
    mark(k, 1, 0);
    if ((rc = build_families(ctx, n, p->delta, false))) return rc;
    mark(k, 1, 1);
    mark(k, 4, 0);
    double* hist = nullptr;
    if (bond_history) {
      const int have = ctx->hist_n == n ? 1 : 0;
      hist = ctx->hist[ctx->hist_last ^ 1];
      k_hist_map<<<walk_grid(n), 256, 4 * sizeof(int32_t) * (size_t)ctx->max_f, ctx->stream>>>(
          n, ctx->row, ctx->col, ctx->hist_row, ctx->hist_col, have, ctx->max_f, ctx->hist_map);
      HIPCHK(hipGetLastError());
    }
    if ((rc = bond_pass(ctx, S, p, p->dt, true, [&](int b) {
           if (b == 0) return;
           mark(k, 4, 1);
           mark(k, 2, 0);
         }, hist)))
      return rc;
    if (bond_history) {
      k_hist_keep<<<blocks_for(ctx->bond_cap, 256, 4096), 256, 0, ctx->stream>>>(n, ctx->row, ctx->col, ctx->hist_row,
                                                                                 ctx->hist_col);
      HIPCHK(hipGetLastError());
      ctx->hist_last ^= 1;
      ctx->hist_n = n;
    }
    mark(k, 2, 1);
    mark(k, 3, 0);
    if ((rc = gather_pass(ctx, S, p, G_STEP, S->mass, nullptr))) return rc;
    mark(k, 3, 1);
    const int64_t ngb = walk_grid(n);
    k_energy<<<1, 256, 0, ctx->stream>>>(ctx->part + kPartPred, npb, ctx->part + kPartGather, (int)ngb,
                                         ctx->E, ctx->row, n, ctx->ctr);
    HIPCHK(hipGetLastError());
  }
  if ((rc = read_counters(ctx))) return rc;
  fill_report(ctx, n, rep, n_steps);
  add_timings(ctx, timed, rep);
  if ((rc = counters_to_status(ctx))) return rc;
  if (p->energy_check && n_steps > 0) {
    double E[3];
    HIPCHK(hipMemcpyAsync(E, ctx->E, sizeof(E), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double mx = std::fmax(std::fabs(E[0]), std::fmax(std::fabs(E[1]), std::fabs(E[2])));
    if (std::fabs(E[0] + E[2] - E[1]) > p->energy_tol * mx)
      return fail(ctx, ULPPM_E_ENERGY, "energy balance (Eq. 69) violated");
  }
  return ULPPM_OK;
}

}  // extern "C"
