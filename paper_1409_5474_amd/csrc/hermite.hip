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
#include "hermite_step.h"

namespace nb {
namespace {

constexpr int kB = 256;
constexpr int kSchedPerThread = 4;
constexpr int kSchedBlock = kB * kSchedPerThread;  // particles per block of the energy sums
// The scheduler's passes take ppt particles per thread: the smallest power of
// two that keeps the block table within kSchedMaxBlocks entries (every block
// of the second pass reads the whole table), so that small systems still
// spread over many compute units.
constexpr int kSchedMaxBlocks = 1024;
inline int sched_ppt(int64_t n) {
  int p = 1;
  while ((n + (int64_t)kB * p - 1) / ((int64_t)kB * p) > kSchedMaxBlocks) p <<= 1;
  return p;
}

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
    const double a1[3] = {acc1[3 * k], acc1[3 * k + 1], acc1[3 * k + 2]};
    const double j1[3] = {jerk1[3 * k], jerk1[3 * k + 1], jerk1[3 * k + 2]};
    correct_particle(i, a1, j1, pos_p, vel_p, pos, vel, acc, jerk, t_tick, level, eta, dt_max, max_level,
                     clamp_dev);
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
// Two deterministic passes, no atomics.  Pass 1: per block, the minimum of
// t_i + dt_i and how many of its particles reach that minimum.  Pass 2: every
// block takes the global minimum t_next from the block table, its offset as
// the counts of the earlier blocks whose minimum is t_next, writes the
// indices of its particles due at t_next in ascending order, and (when
// given the arrays) predicts all its particles to t_next -- the predictor
// reads what the scheduler's pass already has at hand, so it costs no
// launch of its own.
__device__ __forceinline__ int64_t t_end_of(const int64_t* t_tick, const int32_t* level, int64_t i, int max_level) {
  return t_tick[i] + ((int64_t)1 << (max_level - level[i]));
}

// x_p, v_p at t_next of the particles [base, base + count) (below n), one
// thread per component so that every array is read with unit stride; the
// formulas of k_predict.
__device__ __forceinline__ void predict_range(const PredictArgs& p, const int64_t* t_tick, int64_t base,
                                              int64_t count, int64_t n, int64_t t_next, int threads) {
  const int64_t e_end = 3 * (base + count < n ? base + count : n);
  for (int64_t e = 3 * base + threadIdx.x; e < e_end; e += threads) {
    const int64_t i = e / 3;
    const double d = (double)(t_next - t_tick[i]) * p.dt_min;
    const double x = p.pos[e], v = p.vel[e], a = p.acc[e], j = p.jerk[e];
    p.pos_p[e] = x + d * (v + d * (0.5 * a + d * (j * (1.0 / 6.0))));
    p.vel_p[e] = v + d * (a + d * (0.5 * j));
  }
}

// Minimum and sum over the NT threads of a block: shuffles within each
// wavefront, then the wavefront results through LDS (two barriers; the
// second frees wbuf for the next call).  Both are exact, so their order is
// immaterial.
template <int NT>
__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t* wbuf) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t u = __shfl_xor(v, o, 64);
    v = u < v ? u : v;
  }
  if ((threadIdx.x & 63) == 0) wbuf[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t r = wbuf[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) r = wbuf[w] < r ? wbuf[w] : r;
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t* wbuf) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) wbuf[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t r = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) r += wbuf[w];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kB) void k_sched_minc(const int64_t* __restrict__ t_tick,
                                                   const int32_t* __restrict__ level, int64_t n, int max_level,
                                                   int ppt, int64_t* __restrict__ block_min,
                                                   int32_t* __restrict__ block_cnt) {
  __shared__ int64_t wbuf[kB / 64];
  int64_t m = INT64_MAX;
  const int64_t base = (int64_t)blockIdx.x * kB * ppt;
  for (int r = 0; r < ppt; ++r) {
    const int64_t i = base + r * kB + threadIdx.x;
    const int64_t te = i < n ? t_end_of(t_tick, level, i, max_level) : INT64_MAX;
    m = te < m ? te : m;
  }
  const int64_t bm = block_min_i64<kB>(m, wbuf);
  int64_t c = 0;
  for (int r = 0; r < ppt; ++r) {
    const int64_t i = base + r * kB + threadIdx.x;
    c += (i < n && t_end_of(t_tick, level, i, max_level) == bm) ? 1 : 0;
  }
  const int64_t bc = block_sum_i64<kB>(c, wbuf);
  if (threadIdx.x == 0) {
    block_min[blockIdx.x] = bm;
    block_cnt[blockIdx.x] = (int32_t)bc;
  }
}

__global__ __launch_bounds__(kB) void k_sched_write(const int64_t* __restrict__ t_tick,
                                                    const int32_t* __restrict__ level, int64_t n, int max_level,
                                                    int ppt, const int64_t* __restrict__ block_min,
                                                    const int32_t* __restrict__ block_cnt, int nblk,
                                                    int32_t* __restrict__ active, int64_t* __restrict__ sched,
                                                    int32_t* __restrict__ n_active32, int64_t t_stop_host,
                                                    const int64_t* __restrict__ t_stop_dev, PredictArgs pred) {
  __shared__ int64_t wbuf[kB / 64];
  __shared__ int wc[kB / 64];
  // the global minimum, then this block's offset (earlier blocks reaching
  // it); both exact, so independent of the order of the partial results
  int64_t m = INT64_MAX;
  for (int b = threadIdx.x; b < nblk; b += kB) m = block_min[b] < m ? block_min[b] : m;
  const int64_t t_next = block_min_i64<kB>(m, wbuf);
  const bool last_block = blockIdx.x == (unsigned)(nblk - 1);
  int64_t part = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kB)
    if (block_min[b] == t_next) part += block_cnt[b];
  int64_t off = block_sum_i64<kB>(part, wbuf);
  const int64_t base = (int64_t)blockIdx.x * kB * ppt;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < ppt; ++r) {
    const int64_t i = base + r * kB + threadIdx.x;
    const bool flag = i < n && t_end_of(t_tick, level, i, max_level) == t_next;
    // rank among the flagged lanes of the wavefront, then the wavefronts in order
    const uint64_t mask = __ballot(flag);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    __syncthreads();
    if (lane == 0) wc[wave] = __popcll(mask);
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < kB / 64; ++w) {
      before += w < wave ? wc[w] : 0;
      total += wc[w];
    }
    if (flag) active[off + before + rank] = (int32_t)i;
    off += total;
  }
  if (pred.pos) predict_range(pred, t_tick, base, (int64_t)kB * ppt, n, t_next, kB);
  if (last_block && threadIdx.x == 0) {
    // past the stop time the step is empty: every later kernel does nothing
    const int64_t t_stop = t_stop_dev ? *t_stop_dev : t_stop_host;
    const int64_t cnt = t_next <= t_stop ? off : 0;
    sched[0] = t_next;
    sched[1] = cnt;
    if (n_active32) *n_active32 = (int32_t)cnt;
  }
}

// Small systems: one workgroup does both passes (a launch costs more than
// the passes themselves below a few thousand particles).  Same t_next, same
// ascending active list, same predicted state as the two-kernel form.
constexpr int kSchedSingleThreads = 1024;
constexpr int64_t kSchedSingleMax = 16384;

__global__ __launch_bounds__(kSchedSingleThreads) void k_sched_single(const int64_t* __restrict__ t_tick,
                                                                      const int32_t* __restrict__ level, int64_t n,
                                                                      int max_level, int32_t* __restrict__ active,
                                                                      int64_t* __restrict__ sched,
                                                                      int32_t* __restrict__ n_active32,
                                                                      int64_t t_stop_host,
                                                                      const int64_t* __restrict__ t_stop_dev,
                                                                      PredictArgs pred) {
  constexpr int W = kSchedSingleThreads / 64;
  __shared__ int64_t wbuf[W];
  __shared__ int wc[W];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int64_t m = INT64_MAX;
  for (int64_t i = t; i < n; i += kSchedSingleThreads) {
    const int64_t te = t_end_of(t_tick, level, i, max_level);
    m = te < m ? te : m;
  }
  const int64_t t_next = block_min_i64<kSchedSingleThreads>(m, wbuf);
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
  if (pred.pos) {
    predict_range(pred, t_tick, 0, n, n, t_next, kSchedSingleThreads);
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

int schedule_blocks(int64_t n) {
  const int64_t sb = (int64_t)kB * sched_ppt(n);
  return (int)((n + sb - 1) / sb);
}

hipError_t launch_schedule(const int64_t* t_tick, const int32_t* level, int64_t n, int max_level, int32_t* active,
                           int64_t* sched, int64_t* block_min, int32_t* block_cnt, int32_t* n_active32,
                           int64_t t_stop, const int64_t* t_stop_dev, hipStream_t st, const PredictArgs* pred) {
  const PredictArgs p = pred ? *pred : PredictArgs{};
  if (n <= kSchedSingleMax) {
    hipLaunchKernelGGL(k_sched_single, dim3(1), dim3(kSchedSingleThreads), 0, st, t_tick, level, n, max_level,
                       active, sched, n_active32, t_stop, t_stop_dev, p);
    return hipGetLastError();
  }
  const int nblk = schedule_blocks(n);
  const int ppt = sched_ppt(n);
  hipLaunchKernelGGL(k_sched_minc, dim3(nblk), dim3(kB), 0, st, t_tick, level, n, max_level, ppt, block_min,
                     block_cnt);
  hipLaunchKernelGGL(k_sched_write, dim3(nblk), dim3(kB), 0, st, t_tick, level, n, max_level, ppt, block_min,
                     block_cnt, nblk, active, sched, n_active32, t_stop, t_stop_dev, p);
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
