// Force kernel of the sixth-order Hermite scheme (the higher-order Hermite
// integrators that the paper cites for the direct method, section
// "Simulating Collisional systems with direct force evaluation methods"):
// acceleration, jerk, snap and potential of an active i-set in the field of
// all j-particles, each particle moving with its own predicted position,
// velocity and acceleration.  For r = x_j - x_i, u = v_j - v_i,
// w = a_j - a_i, s = |r|^2 + eps2, q = s^{-1/2}:
//   alpha = (r.u) q^2,  beta = (u.u + r.w) q^2 + alpha^2
//   A = m q^3 r,  J = m q^3 u - 3 alpha A,  S = m q^3 w - 6 alpha J - 3 beta A,
//   phi -= m q
// (the recursive form of the successive time derivatives of m r s^{-3/2}).
//
// All arithmetic is double precision.  Layout as the LDS path of the
// fourth-order kernel: j-tiles of kTile particles staged in LDS as five
// double2 streams (x y | z m | vx vy | vz ax | ay az), one i-particle per
// lane, the j-range cut into S chunks over a persistent grid, per-tile
// double sums folded into a compensated (TwoSum) accumulator, and a second
// kernel adding the S partial blocks in a fixed order.  The active count may
// be read from device memory, so a block step can be captured in a graph.
// The self pair is kept in the loop (it adds exactly zero to A, J and S) and
// its potential term is removed with the identical value; with eps2 == 0
// every pair at zero distance is dropped instead.
#include <map>
#include <mutex>

#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kWG6 = 256;   // threads per workgroup = i-particles per block
constexpr int kT6 = 256;    // j-particles per staged tile
constexpr int kC6 = 10;     // acc, jerk, snap, pot

// v_rsq_f64 is accurate to about 2^-24; one third-order Newton step
// y <- y (1 + e/2 + 3 e^2/8), e = 1 - s y^2, brings it to double rounding.
__device__ __forceinline__ double rsqrt6(double s) {
  const double y = __builtin_amdgcn_rsq(s);
  const double e = fma(-(s * y), y, 1.0);
  return fma(y, e * fma(e, 0.375, 0.5), y);
}

// hi + lo += x without losing the low part (Knuth's TwoSum).
__device__ __forceinline__ void two_sum6(double& hi, double& lo, double x) {
  const double s = hi + x;
  const double bp = s - hi;
  const double err = (hi - (s - bp)) + (x - bp);
  hi = s;
  lo += err;
}

// Chunks per i-block: enough (i-block, chunk) items to fill the chip, each
// chunk at least one tile.
__host__ __device__ inline int split6(int64_t n_act, int target_items, int64_t n) {
  const int64_t n_iblk = (n_act + kWG6 - 1) / kWG6;
  if (n_iblk <= 0) return 1;
  int64_t s = (target_items + n_iblk - 1) / n_iblk;
  const int64_t max_s = (n + kT6 - 1) / kT6;
  if (s > max_s) s = max_s;
  if (s < 1) s = 1;
  return (int)s;
}

__host__ __device__ inline int64_t chunk6(int64_t n, int S) {
  const int64_t per = (n + S - 1) / S;
  return ((per + kT6 - 1) / kT6) * kT6;
}

struct Tile6 {
  double2 xy[kT6];
  double2 zm[kT6];
  double2 vxy[kT6];
  double2 vza[kT6];   // vz, ax
  double2 ayz[kT6];   // ay, az
};

template <bool MASK>
__device__ __forceinline__ void pair6(const double* I, double2 xy, double2 zm, double2 vxy, double2 vza,
                                      double2 ayz, double e2, double* T) {
  const double rx = xy.x - I[0], ry = xy.y - I[1], rz = zm.x - I[2];
  const double ux = vxy.x - I[3], uy = vxy.y - I[4], uz = vza.x - I[5];
  const double wx = vza.y - I[6], wy = ayz.x - I[7], wz = ayz.y - I[8];
  const double s = fma(rz, rz, fma(ry, ry, fma(rx, rx, e2)));
  double q = rsqrt6(s);
  if (MASK) q = (s > 0.0) ? q : 0.0;
  const double q2 = q * q;
  const double ru = fma(rz, uz, fma(ry, uy, rx * ux));
  const double uu = fma(uz, uz, fma(uy, uy, ux * ux));
  const double rw = fma(rz, wz, fma(ry, wy, rx * wx));
  const double alpha = ru * q2;
  const double beta = fma(alpha, alpha, (uu + rw) * q2);
  const double mq = zm.y * q;
  const double mq3 = mq * q2;
  const double ax = mq3 * rx, ay = mq3 * ry, az = mq3 * rz;
  const double a3 = -3.0 * alpha;
  const double jx = fma(a3, ax, mq3 * ux), jy = fma(a3, ay, mq3 * uy), jz = fma(a3, az, mq3 * uz);
  const double a6 = -6.0 * alpha, b3 = -3.0 * beta;
  T[0] += ax; T[1] += ay; T[2] += az;
  T[3] += jx; T[4] += jy; T[5] += jz;
  T[6] += fma(b3, ax, fma(a6, jx, mq3 * wx));
  T[7] += fma(b3, ay, fma(a6, jy, mq3 * wy));
  T[8] += fma(b3, az, fma(a6, jz, mq3 * wz));
  T[9] += mq;
}

template <bool MASK>
__device__ __forceinline__ void item6(Tile6& tile, const Force6Args& a, int64_t jbeg, int64_t jend, int64_t n_act,
                                      int64_t k0, bool final_out, double* part) {
  const int t = threadIdx.x;
  const int64_t k = k0 + t;
  int64_t irow = k < n_act ? (int64_t)a.active[k] : -1;
  if (k < n_act && !row_in_range(irow, 0, a.n)) {  // not a particle: skipped, and reported by nb_sync
    if (a.err) atomicOr(a.err, kErrActiveRange);
    irow = -1;
  }
  const int64_t ir = irow >= 0 ? irow : 0;
  double I[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    I[c] = a.pos[3 * ir + c];
    I[3 + c] = a.vel[3 * ir + c];
    I[6 + c] = a.accj[3 * ir + c];
  }
  const double e2 = a.eps2;
  double hi[kC6], lo[kC6], T[kC6];
#pragma unroll
  for (int c = 0; c < kC6; ++c) hi[c] = lo[c] = T[c] = 0.0;

  for (int64_t base = jbeg; base < jend; base += kT6) {
    __syncthreads();  // every lane is done with the previous tile
    {
      const int64_t j = base + t;
      const bool ok = j < jend;
      const int64_t jr = ok ? j : 0;
      tile.xy[t] = ok ? make_double2(a.pos[3 * jr], a.pos[3 * jr + 1]) : make_double2(0.0, 0.0);
      tile.zm[t] = ok ? make_double2(a.pos[3 * jr + 2], a.mass[jr]) : make_double2(0.0, 0.0);
      tile.vxy[t] = ok ? make_double2(a.vel[3 * jr], a.vel[3 * jr + 1]) : make_double2(0.0, 0.0);
      tile.vza[t] = ok ? make_double2(a.vel[3 * jr + 2], a.accj[3 * jr]) : make_double2(0.0, 0.0);
      tile.ayz[t] = ok ? make_double2(a.accj[3 * jr + 1], a.accj[3 * jr + 2]) : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 2
    for (int jj = 0; jj < kT6; ++jj)
      pair6<MASK>(I, tile.xy[jj], tile.zm[jj], tile.vxy[jj], tile.vza[jj], tile.ayz[jj], e2, T);
#pragma unroll
    for (int c = 0; c < kC6; ++c) {
      two_sum6(hi[c], lo[c], T[c]);
      T[c] = 0.0;
    }
  }
  if (irow < 0) return;
  double v[kC6];
#pragma unroll
  for (int c = 0; c < kC6; ++c) v[c] = hi[c] + lo[c];
  if (final_out) {
    const double self = (e2 > 0.0) ? a.mass[irow] * rsqrt6(e2) : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.acc[3 * k + c] = v[c];
      a.jerk[3 * k + c] = v[3 + c];
      a.snap[3 * k + c] = v[6 + c];
    }
    a.pot[k] = -(v[9] - self);
  } else {
#pragma unroll
    for (int c = 0; c < kC6; ++c) part[c * n_act + k] = v[c];
  }
}

__device__ __forceinline__ int64_t active_count6(const Force6Args& a) {
  int64_t n_act = a.n_active;
  if (a.n_active_dev) {
    const int64_t d = *a.n_active_dev;
    n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
  }
  return n_act;
}

template <bool MASK>
__global__ __launch_bounds__(kWG6) void k_forces6(Force6Args a) {
  __shared__ Tile6 tile;
  const int64_t n_act = active_count6(a);
  const int S = a.n_active_dev ? split6(n_act, a.target_items, a.n) : a.S;
  const int64_t n_iblk = (n_act + kWG6 - 1) / kWG6;
  const int64_t items = n_iblk * S;
  const int64_t clen = chunk6(a.n, S);
  for (int64_t w = blockIdx.x; w < items; w += gridDim.x) {
    const int64_t chunk = w / n_iblk;
    const int64_t iblk = w - chunk * n_iblk;
    const int64_t jb = chunk * clen;
    const int64_t je = jb + clen < a.n ? jb + clen : a.n;
    item6<MASK>(tile, a, jb, je, n_act, iblk * kWG6, S == 1, a.part + chunk * kC6 * n_act);
  }
}

// Fixed-order sum of the S partial blocks, self-term removal, output.
__global__ __launch_bounds__(256) void k_reduce6(Force6Args a) {
  const int64_t n_act = active_count6(a);
  const int S = a.n_active_dev ? split6(n_act, a.target_items, a.n) : a.S;
  if (S <= 1) return;
  const int64_t total = kC6 * n_act;
  const int g = chunk_lanes(S);
  const int lg = __builtin_ctz(g);
  const int lane = threadIdx.x & (g - 1);
  for (int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> lg; idx < total;
       idx += ((int64_t)gridDim.x * blockDim.x) >> lg) {
    const int64_t c = idx / n_act;
    const int64_t k = idx - c * n_act;
    const double s = sum_blocks(a.part + c * n_act + k, kC6 * n_act, S, lane, g);
    if (lane != 0) continue;
    if (!row_in_range(a.active[k], 0, a.n)) continue;  // skipped row (flagged by the force pass)
    if (c < 3) {
      a.acc[3 * k + c] = s;
    } else if (c < 6) {
      a.jerk[3 * k + c - 3] = s;
    } else if (c < 9) {
      a.snap[3 * k + c - 6] = s;
    } else {
      const double self = (a.eps2 > 0.0) ? a.mass[a.active[k]] * rsqrt6(a.eps2) : 0.0;
      a.pot[k] = -(s - self);
    }
  }
}

}  // namespace

int forces6_resident_wgs(bool mask) {
  static std::mutex mu;
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(mask ? 1 : 0);
  if (it != cache.end()) return it->second;
  int nblk = 0;
  const void* fn = mask ? (const void*)k_forces6<true> : (const void*)k_forces6<false>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, fn, kWG6, 0) != hipSuccess || nblk < 1) {
    (void)hipGetLastError();
    nblk = 1;
  }
  cache[mask ? 1 : 0] = nblk;
  return nblk;
}

int forces6_split(int64_t n_act, int target_items, int64_t n) { return split6(n_act, target_items, n); }

int64_t forces6_workspace_rows(int64_t n_max, int target_items, int64_t n) {
  // S * n_act over every count up to n_max: S <= target / n_iblk + 1, so
  // S * n_act <= (target + n_iblk) * kWG6 <= target * kWG6 + n_max + kWG6
  const int64_t bound = (int64_t)target_items * kWG6 + n_max + kWG6;
  const int64_t max_s = (n + kT6 - 1) / kT6;
  return bound < max_s * n_max ? bound : max_s * n_max;
}

hipError_t launch_forces6(const Force6Args& a, bool mask, int grid, hipStream_t st) {
  if (grid < 1) grid = 1;
  if (mask)
    hipLaunchKernelGGL(k_forces6<true>, dim3(grid), dim3(kWG6), 0, st, a);
  else
    hipLaunchKernelGGL(k_forces6<false>, dim3(grid), dim3(kWG6), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!a.n_active_dev && a.S <= 1) return hipSuccess;
  // threads: the outputs times the lanes per output (with the count on the
  // device, as for the fourth-order reduce: up to 1024 blocks, at least the
  // outputs' threads)
  const int64_t outs = kC6 * a.n_active;
  int64_t threads = outs * chunk_lanes(a.S);
  if (a.n_active_dev) {
    threads = outs * 64 < (int64_t)1024 * 256 ? outs * 64 : (int64_t)1024 * 256;
    if (threads < outs) threads = outs;
  }
  int64_t rg = (threads + 255) / 256;
  if (rg > 4096) rg = 4096;
  if (rg < 1) rg = 1;
  hipLaunchKernelGGL(k_reduce6, dim3((int)rg), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace nb
