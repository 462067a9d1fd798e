// Hermite block-step kernels: predictor, corrector with the Aarseth step
// criterion and power-of-two levels, start-up levels, block scheduler and
// the energy/momentum sums.  All of them are HBM-bound element-wise passes
// or small reductions; the arithmetic is IEEE double throughout.
//
// The integrator is the 4th-order Hermite predictor-corrector with block
// time steps that the paper names for its direct code (sections
// "Simulating Collisional systems with direct force evaluation methods":
// block time steps make the i-particle parallelisation possible; and
// "Simulating galaxy mergers with supermassive black holes": ph4).  The
// paper gives no formulas; the library follows the Makino-Aarseth form
// described in nbody.h.
#include "nb_internal.h"

namespace nb {
namespace {

constexpr int kB = 256;
constexpr int kSchedPerThread = 4;
constexpr int kSchedBlock = kB * kSchedPerThread;  // particles per scheduler block

// ---------------------------------------------------------------- predict --
// One thread per (particle, component): every array is read with unit
// stride.  d = (t_next - t_i) dt_min is exact (integer ticks times a power
// of two times dt_max).
__global__ __launch_bounds__(kB) void k_predict(const double* __restrict__ pos, const double* __restrict__ vel,
                                                const double* __restrict__ acc, const double* __restrict__ jerk,
                                                const int64_t* __restrict__ t_tick, int64_t t_next_host,
                                                const int64_t* __restrict__ t_next_dev, double dt_min, int64_t n3,
                                                double* __restrict__ pos_p, double* __restrict__ vel_p) {
  const int64_t t_next = t_next_dev ? *t_next_dev : t_next_host;
  for (int64_t e = (int64_t)blockIdx.x * kB + threadIdx.x; e < n3; e += (int64_t)gridDim.x * kB) {
    const int64_t i = e / 3;
    const double d = (double)(t_next - t_tick[i]) * dt_min;
    const double x = pos[e], v = vel[e], a = acc[e], j = jerk[e];
    pos_p[e] = x + d * (v + d * (0.5 * a + d * (j * (1.0 / 6.0))));
    vel_p[e] = v + d * (a + d * (0.5 * j));
  }
}

__device__ __forceinline__ double norm3(double x, double y, double z) { return sqrt(x * x + y * y + z * z); }

// ---------------------------------------------------------------- correct --
__global__ __launch_bounds__(kB) void k_correct(const int32_t* __restrict__ active, int64_t n_active_host,
                                                const int64_t* __restrict__ n_active_dev, int64_t n_rows,
                                                unsigned int* __restrict__ err,
                                                const double* __restrict__ pos_p, const double* __restrict__ vel_p,
                                                const double* __restrict__ acc1, const double* __restrict__ jerk1,
                                                double* __restrict__ pos, double* __restrict__ vel,
                                                double* __restrict__ acc, double* __restrict__ jerk,
                                                int64_t* __restrict__ t_tick, int32_t* __restrict__ level,
                                                double eta, double dt_max, int max_level,
                                                unsigned long long* __restrict__ clamp_dev,
                                                unsigned long long* __restrict__ step_dev) {
  int64_t n_act = n_active_host;
  if (n_active_dev) {
    const int64_t d = *n_active_dev;
    n_act = d < n_act ? (d < 0 ? 0 : d) : n_act;
  }
  if (step_dev && n_act > 0 && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(step_dev, 1ull);
  for (int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x; k < n_act; k += (int64_t)gridDim.x * kB) {
    const int64_t i = active[k];
    if (!row_in_range(i, 0, n_rows)) {  // not a particle: skipped, and reported by nb_sync
      if (err) atomicOr(err, kErrActiveRange);
      continue;
    }
    const int L = level[i];
    const double dt = ldexp(dt_max, -L);
    const double dt2 = dt * dt, dt3 = dt2 * dt;
    double a1[3], j1[3], a2[3], a3[3], a2e[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double a0 = acc[3 * i + c], j0 = jerk[3 * i + c];
      a1[c] = acc1[3 * k + c];
      j1[c] = jerk1[3 * k + c];
      a2[c] = (-6.0 * (a0 - a1[c]) - dt * (4.0 * j0 + 2.0 * j1[c])) / dt2;
      a3[c] = (12.0 * (a0 - a1[c]) + 6.0 * dt * (j0 + j1[c])) / dt3;
      const double dt4 = dt2 * dt2;
      pos[3 * i + c] = pos_p[3 * i + c] + a2[c] * (dt4 / 24.0) + a3[c] * (dt4 * dt / 120.0);
      vel[3 * i + c] = vel_p[3 * i + c] + a2[c] * (dt3 / 6.0) + a3[c] * (dt4 / 24.0);
      acc[3 * i + c] = a1[c];
      jerk[3 * i + c] = j1[c];
      a2e[c] = a2[c] + a3[c] * dt;
    }
    const double na1 = norm3(a1[0], a1[1], a1[2]);
    const double nj1 = norm3(j1[0], j1[1], j1[2]);
    const double na2 = norm3(a2e[0], a2e[1], a2e[2]);
    const double na3 = norm3(a3[0], a3[1], a3[2]);
    const double num = na1 * na2 + nj1 * nj1;
    const double den = nj1 * na3 + na2 * na2;
    const double ds = den > 0.0 ? sqrt(eta * num / den) : dt_max;
    const int64_t t_new = t_tick[i] + ((int64_t)1 << (max_level - L));
    int Ln = L;
    double dtc = dt;
    if (ds < dtc) {
      while (dtc > ds && Ln < max_level) {
        ++Ln;
        dtc = ldexp(dt_max, -Ln);
      }
      if (dtc > ds && clamp_dev) atomicAdd(clamp_dev, 1ull);
    } else if (ds >= 2.0 * dtc && Ln > 0) {
      const int64_t two_dt = (int64_t)1 << (max_level - Ln + 1);
      if (t_new % two_dt == 0) --Ln;
    }
    t_tick[i] = t_new;
    level[i] = Ln;
  }
}

// ---------------------------------------------------------------- startup --
__global__ __launch_bounds__(kB) void k_startup(const double* __restrict__ acc, const double* __restrict__ jerk,
                                                int64_t n, double eta, double dt_max, int max_level,
                                                int32_t* __restrict__ level) {
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    const double na = norm3(acc[3 * i], acc[3 * i + 1], acc[3 * i + 2]);
    const double nj = norm3(jerk[3 * i], jerk[3 * i + 1], jerk[3 * i + 2]);
    int L = 0;
    if (nj != 0.0) {
      const double target = eta * na / nj;
      while (ldexp(dt_max, -L) > target && L < max_level) ++L;
    }
    level[i] = L;
  }
}

// --------------------------------------------------------------- schedule --
// Three deterministic passes, no atomics: per-block minimum of t_i + dt_i;
// per-block count of particles reaching the global minimum; ordered write
// of their indices (block offset + in-block exclusive scan).
__device__ __forceinline__ int64_t t_end_of(const int64_t* t_tick, const int32_t* level, int64_t i, int max_level) {
  return t_tick[i] + ((int64_t)1 << (max_level - level[i]));
}

__global__ __launch_bounds__(kB) void k_sched_min(const int64_t* __restrict__ t_tick,
                                                  const int32_t* __restrict__ level, int64_t n, int max_level,
                                                  int64_t* __restrict__ block_min) {
  __shared__ int64_t red[kB];
  int64_t m = INT64_MAX;
  const int64_t base = (int64_t)blockIdx.x * kSchedBlock;
  for (int r = 0; r < kSchedPerThread; ++r) {
    const int64_t i = base + r * kB + threadIdx.x;
    if (i < n) {
      const int64_t te = t_end_of(t_tick, level, i, max_level);
      m = te < m ? te : m;
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const int64_t b = red[threadIdx.x + o];
      if (b < red[threadIdx.x]) red[threadIdx.x] = b;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) block_min[blockIdx.x] = red[0];
}

__device__ int64_t global_min(const int64_t* block_min, int nblk, int64_t* red) {
  int64_t m = INT64_MAX;
  for (int b = threadIdx.x; b < nblk; b += kB) m = block_min[b] < m ? block_min[b] : m;
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const int64_t b = red[threadIdx.x + o];
      if (b < red[threadIdx.x]) red[threadIdx.x] = b;
    }
    __syncthreads();
  }
  const int64_t r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kB) void k_sched_count(const int64_t* __restrict__ t_tick,
                                                    const int32_t* __restrict__ level, int64_t n, int max_level,
                                                    const int64_t* __restrict__ block_min, int nblk,
                                                    int32_t* __restrict__ block_cnt, int64_t* __restrict__ sched) {
  __shared__ int64_t red[kB];
  __shared__ int cnt[kB];
  const int64_t t_next = global_min(block_min, nblk, red);
  int c = 0;
  const int64_t base = (int64_t)blockIdx.x * kSchedBlock;
  for (int r = 0; r < kSchedPerThread; ++r) {
    const int64_t i = base + r * kB + threadIdx.x;
    if (i < n && t_end_of(t_tick, level, i, max_level) == t_next) ++c;
  }
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    block_cnt[blockIdx.x] = cnt[0];
    if (blockIdx.x == 0) sched[0] = t_next;
  }
}

__global__ __launch_bounds__(kB) void k_sched_write(const int64_t* __restrict__ t_tick,
                                                    const int32_t* __restrict__ level, int64_t n, int max_level,
                                                    const int32_t* __restrict__ block_cnt, int nblk,
                                                    const int64_t* sched_in,
                                                    int32_t* __restrict__ active, int64_t* sched,
                                                    int32_t* __restrict__ n_active32, int64_t t_stop_host,
                                                    const int64_t* __restrict__ t_stop_dev) {
  __shared__ int sc[kB];
  __shared__ int64_t off_s;
  const int64_t t_next = sched_in[0];
  // offset of this block = sum of the counts of the blocks before it
  int64_t part = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kB) part += block_cnt[b];
  sc[threadIdx.x] = (int)part;
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sc[threadIdx.x] += sc[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) off_s = sc[0];
  __syncthreads();
  int64_t off = off_s;
  const int64_t base = (int64_t)blockIdx.x * kSchedBlock;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < kSchedPerThread; ++r) {
    const int64_t i = base + r * kB + threadIdx.x;
    const bool flag = i < n && t_end_of(t_tick, level, i, max_level) == t_next;
    // rank among the flagged lanes of the wavefront, then the wavefronts in order
    const uint64_t mask = __ballot(flag);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    __syncthreads();
    if (lane == 0) sc[wave] = __popcll(mask);
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < kB / 64; ++w) {
      before += w < wave ? sc[w] : 0;
      total += sc[w];
    }
    if (flag) active[off + before + rank] = (int32_t)i;
    off += total;
  }
  if (blockIdx.x == (unsigned)(nblk - 1) && threadIdx.x == 0) {
    // past the stop time the step is empty: every later kernel does nothing
    const int64_t t_stop = t_stop_dev ? *t_stop_dev : t_stop_host;
    const int64_t cnt = t_next <= t_stop ? off : 0;
    sched[1] = cnt;
    if (n_active32) *n_active32 = (int32_t)cnt;
  }
}

// Small systems: one workgroup does all three passes (a launch costs more
// than the passes themselves below a few thousand particles).  Same t_next,
// same ascending active list as the three-kernel form.
constexpr int kSchedSingleThreads = 1024;
constexpr int64_t kSchedSingleMax = 16384;

__global__ __launch_bounds__(kSchedSingleThreads) void k_sched_single(const int64_t* __restrict__ t_tick,
                                                                      const int32_t* __restrict__ level, int64_t n,
                                                                      int max_level, int32_t* __restrict__ active,
                                                                      int64_t* __restrict__ sched,
                                                                      int32_t* __restrict__ n_active32,
                                                                      int64_t t_stop_host,
                                                                      const int64_t* __restrict__ t_stop_dev) {
  constexpr int W = kSchedSingleThreads / 64;
  __shared__ int64_t red[kSchedSingleThreads];
  __shared__ int wc[W];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int64_t m = INT64_MAX;
  for (int64_t i = t; i < n; i += kSchedSingleThreads) {
    const int64_t te = t_end_of(t_tick, level, i, max_level);
    m = te < m ? te : m;
  }
  red[t] = m;
  __syncthreads();
  for (int o = kSchedSingleThreads / 2; o > 0; o >>= 1) {
    if (t < o && red[t + o] < red[t]) red[t] = red[t + o];
    __syncthreads();
  }
  const int64_t t_next = red[0];
  int64_t off = 0;
  for (int64_t base = 0; base < n; base += kSchedSingleThreads) {
    const int64_t i = base + t;
    const bool flag = i < n && t_end_of(t_tick, level, i, max_level) == t_next;
    const uint64_t mask = __ballot(flag);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    __syncthreads();
    if (lane == 0) wc[wave] = __popcll(mask);
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < W; ++w) {
      before += w < wave ? wc[w] : 0;
      total += wc[w];
    }
    if (flag) active[off + before + rank] = (int32_t)i;
    off += total;
  }
  if (t == 0) {
    const int64_t t_stop = t_stop_dev ? *t_stop_dev : t_stop_host;
    const int64_t cnt = t_next <= t_stop ? off : 0;
    sched[0] = t_next;
    sched[1] = cnt;
    if (n_active32) *n_active32 = (int32_t)cnt;
  }
}

// ----------------------------------------------------------------- energy --
// Per-block sums of K, m phi, m v, m x cross v (tree order), then one block
// adds the block sums in index order.
__global__ __launch_bounds__(kB) void k_energy_part(const double* __restrict__ pos, const double* __restrict__ vel,
                                                    const double* __restrict__ mass, const double* __restrict__ pot,
                                                    int64_t n, double* __restrict__ part) {
  __shared__ double red[8][kB];
  double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t base = (int64_t)blockIdx.x * kSchedBlock;
  for (int r = 0; r < kSchedPerThread; ++r) {
    const int64_t i = base + r * kB + threadIdx.x;
    if (i < n) {
      const double m = mass[i];
      const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
      const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
      q[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
      q[1] += 0.5 * m * pot[i];
      q[2] += m * vx; q[3] += m * vy; q[4] += m * vz;
      q[5] += m * (y * vz - z * vy);
      q[6] += m * (z * vx - x * vz);
      q[7] += m * (x * vy - y * vx);
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) red[c][threadIdx.x] = q[c];
  __syncthreads();
  for (int o = kB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
#pragma unroll
      for (int c = 0; c < 8; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x < 8) part[(int64_t)blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// Fixed-order sum of the block partials: thread (c, l) of 8 x 32 adds the
// partials l, l + 32, ... of component c (consecutive threads read
// consecutive words) into four running sums taken in turn, so four loads are
// in flight; then each component's 32 sums are added pairwise.
__global__ __launch_bounds__(kB) void k_energy_final(const double* __restrict__ part, int nblk,
                                                     double* __restrict__ out) {
  __shared__ double red[8][33];
  const int c = threadIdx.x & 7, l = threadIdx.x >> 3;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int b = l;
  for (; b + 96 < nblk; b += 128) {
    s0 += part[(int64_t)b * 8 + c];
    s1 += part[(int64_t)(b + 32) * 8 + c];
    s2 += part[(int64_t)(b + 64) * 8 + c];
    s3 += part[(int64_t)(b + 96) * 8 + c];
  }
  for (; b < nblk; b += 32) s0 += part[(int64_t)b * 8 + c];
  red[c][l] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  for (int o = 16; o > 0; o >>= 1) {
    if (l < o) red[c][l] += red[c][l + o];
    __syncthreads();
  }
  if (threadIdx.x < 8) out[threadIdx.x] = red[threadIdx.x][0];
}

inline int grid_for(int64_t work, int cap) {
  int64_t g = (work + kB - 1) / kB;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_predict(const double* pos, const double* vel, const double* acc, const double* jerk,
                          const int64_t* t_tick, int64_t t_next, const int64_t* t_next_dev, double dt_min, int64_t n,
                          double* pos_p, double* vel_p, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_predict, dim3(grid_for(3 * n, 32768)), dim3(kB), 0, st, pos, vel, acc, jerk, t_tick, t_next,
                     t_next_dev, dt_min, 3 * n, pos_p, vel_p);
  return hipGetLastError();
}

hipError_t launch_correct(const int32_t* active, int64_t n_active, const int64_t* n_active_dev, int64_t n_rows,
                          unsigned int* err, const double* pos_p, const double* vel_p, const double* acc1,
                          const double* jerk1, double* pos, double* vel, double* acc, double* jerk,
                          int64_t* t_tick, int32_t* level, double eta, double dt_max, int max_level,
                          int64_t* clamp_dev, hipStream_t st) {
  if (n_active <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_correct, dim3(grid_for(n_active, 16384)), dim3(kB), 0, st, active, n_active, n_active_dev,
                     n_rows, err, pos_p, vel_p, acc1, jerk1, pos, vel, acc, jerk, t_tick, level, eta, dt_max, max_level,
                     reinterpret_cast<unsigned long long*>(clamp_dev), nullptr);
  return hipGetLastError();
}

hipError_t launch_correct_step(const int32_t* active, int64_t n_max, const int64_t* n_active_dev, int64_t n_rows,
                               unsigned int* err, const double* pos_p, const double* vel_p, const double* acc1,
                               const double* jerk1, double* pos, double* vel, double* acc, double* jerk,
                               int64_t* t_tick, int32_t* level, double eta, double dt_max, int max_level,
                               int64_t* clamp_dev, int64_t* step_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_correct, dim3(grid_for(n_max, 1024)), dim3(kB), 0, st, active, n_max, n_active_dev, n_rows,
                     err, pos_p,
                     vel_p, acc1, jerk1, pos, vel, acc, jerk, t_tick, level, eta, dt_max, max_level,
                     reinterpret_cast<unsigned long long*>(clamp_dev),
                     reinterpret_cast<unsigned long long*>(step_dev));
  return hipGetLastError();
}

hipError_t launch_startup(const double* acc, const double* jerk, int64_t n, double eta, double dt_max, int max_level,
                          int32_t* level, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_startup, dim3(grid_for(n, 4096)), dim3(kB), 0, st, acc, jerk, n, eta, dt_max, max_level,
                     level);
  return hipGetLastError();
}

int schedule_blocks(int64_t n) { return (int)((n + kSchedBlock - 1) / kSchedBlock); }

hipError_t launch_schedule(const int64_t* t_tick, const int32_t* level, int64_t n, int max_level, int32_t* active,
                           int64_t* sched, int64_t* block_min, int32_t* block_cnt, int32_t* n_active32,
                           int64_t t_stop, const int64_t* t_stop_dev, hipStream_t st) {
  if (n <= kSchedSingleMax) {
    hipLaunchKernelGGL(k_sched_single, dim3(1), dim3(kSchedSingleThreads), 0, st, t_tick, level, n, max_level,
                       active, sched, n_active32, t_stop, t_stop_dev);
    return hipGetLastError();
  }
  const int nblk = schedule_blocks(n);
  hipLaunchKernelGGL(k_sched_min, dim3(nblk), dim3(kB), 0, st, t_tick, level, n, max_level, block_min);
  hipLaunchKernelGGL(k_sched_count, dim3(nblk), dim3(kB), 0, st, t_tick, level, n, max_level, block_min, nblk,
                     block_cnt, sched);
  hipLaunchKernelGGL(k_sched_write, dim3(nblk), dim3(kB), 0, st, t_tick, level, n, max_level, block_cnt, nblk,
                     sched, active, sched, n_active32, t_stop, t_stop_dev);
  return hipGetLastError();
}

int energy_blocks(int64_t n) { return (int)((n + kSchedBlock - 1) / kSchedBlock); }

hipError_t launch_energy(const double* pos, const double* vel, const double* mass, const double* pot, int64_t n,
                         double* part, double* out, hipStream_t st) {
  const int nblk = energy_blocks(n);
  hipLaunchKernelGGL(k_energy_part, dim3(nblk), dim3(kB), 0, st, pos, vel, mass, pot, n, part);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kB), 0, st, part, nblk, out);
  return hipGetLastError();
}

}  // namespace nb
